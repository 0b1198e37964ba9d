// Kernel argument blocks and launcher declarations shared by the kernel
// translation units and the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "fpc_collide.h"

namespace fpc {

// One outer face of the box as the kernels see it.
struct FaceDev {
  int wall;             // 1: wall rules apply; 0: periodic
  int lid;              // moving wall for f
  int dirichlet;        // anti-bounce-back for g
  double Tw;            // uniform wall temperature
  const double* Tprof;  // optional per-node wall temperature (tangential axes, slower first)
  double uw[3];         // wall velocity
};

template <class R>
struct StepArgs {
  const R* __restrict__ src;  // S_{n-1}
  R* __restrict__ dst;        // S_n
  int nx, ny, nz;
  int nxp;                    // row length of the storage layout (nx rounded up to 64)
  int per[3];                 // axis periodic flags
  CollParams<R> c;
  R rho_w;                    // moving-wall density
  // storage reference of g: Tr(x, y, z) = T_o + Tg . (x, y, z)
  // (uniform: T_o = c.T_r, Tg = 0)
  R T_o;
  R Tg[3];
  FaceDev face[6];
};

// FP32 storage holds deviations from the references; FP64 storage holds the
// plain populations (references zero), so the FP64 kernels compile them out.
template <class R>
constexpr bool kDeviations = sizeof(R) == 4;

// Storage reference of the thermal populations at node (x, y, z).
template <class R>
__device__ __forceinline__ R tref(const StepArgs<R>& a, int x, int y, int z) {
  if constexpr (!kDeviations<R>) return R(0);
  return a.T_o + (a.Tg[0] * R(x) + a.Tg[1] * R(y) + a.Tg[2] * R(z));
}
// XCD-aware block order.  Workgroups are dispatched to the 8 XCDs round-robin
// by linear block index, and each XCD has its own L2.  The remap hands XCD k
// the k-th contiguous range of logical blocks, so that neighbouring rows (and
// z planes) are processed by the same XCD and their pulls can hit its L2.
// Returns the logical block coordinates of this workgroup (a bijection).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ dim3 xcd_block() {
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned k = b % kXcds, q = nb / kXcds, r = nb % kXcds;
  const unsigned l = k * q + (k < r ? k : r) + b / kXcds;  // start of XCD k's range + rank within it
  return dim3(l % gridDim.x, (l / gridDim.x) % gridDim.y, l / (gridDim.x * gridDim.y));
}

// The same within each z plane of blocks: XCD k takes the k-th contiguous
// range of the plane's blocks (identity when a plane's block count is not a
// multiple of 8).
__device__ __forceinline__ dim3 xcd_block_plane() {
  const unsigned g = gridDim.x * gridDim.y;
  if (g % kXcds != 0) return dim3(blockIdx.x, blockIdx.y, blockIdx.z);
  const unsigned i = blockIdx.x + gridDim.x * blockIdx.y;  // in-plane index; XCD = i % 8 since g % 8 == 0
  const unsigned l = (i % kXcds) * (g / kXcds) + i / kXcds;
  return dim3(l % gridDim.x, l / gridDim.x, blockIdx.z);
}

// Block order of the step and adjoint kernels (launch tuning, measured):
// contiguous ranges of rows per XCD in 2D; in 3D FP32, contiguous ranges of
// rows per XCD within each z plane; launch order otherwise.
#ifndef FPC_XCD_2D
#define FPC_XCD_2D 1
#endif
#ifndef FPC_XCD_3DF
#define FPC_XCD_3DF 1
#endif
template <int D, int S>
__device__ __forceinline__ dim3 block_order() {
  if (D == 2 && FPC_XCD_2D) return xcd_block();
  if (D == 3 && S == 4 && FPC_XCD_3DF) return xcd_block_plane();
  return dim3(blockIdx.x, blockIdx.y, blockIdx.z);
}

// Launchers of the fused step (defined in fpc_step.hip).
// tk: thermal lattice, 0 = D2Q5 / D3Q7, 1 = D2Q9 / D3Q15 (FP64 only).
// mode: 0 = step (pull from args.src), 1 = init (equilibrium from T_init).
template <class R>
hipError_t launch_step2d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s);
template <class R>
hipError_t launch_step3d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s);

// Adjoint kernels (fpc_adjoint.hip).  `a.src` is S_{n-1} (adjoint step) or
// unused (adjoint of the initial collision).
template <class R>
hipError_t launch_adjoint_step(const StepArgs<R>& a, int dim, int up, const void* lam_in, void* lam_out,
                               const double* dJdT, double ke, double* const dtheta[6], hipStream_t s);
template <class R>
hipError_t launch_adjoint_init(const StepArgs<R>& a, int dim, int up, const double* T_init, const void* lam0,
                               const double* dJdT, double ke, double* dTinit, hipStream_t s);

// Node-level utilities (fpc_kernels_util.hip).
struct StateDesc {
  const void* src;
  int precision;  // 0 FP64, 1 FP32 deviations
  int lattice;    // 1 = 2D, 2 = 3D
  int nx, ny, nz;
  int nxp;  // row length of the storage layout (nx rounded up to 64)
  double rho_r, T_r;  // storage offsets (T_r at the box centre)
  double T_o, Tg[3];  // thermal storage reference Tr(x, y, z) = T_o + Tg . (x, y, z)
  double cs2T;
  double gbeta, T0;
  int up;
};

hipError_t launch_macros(const StateDesc& d, double* rho, double* u, double* T, hipStream_t s);
hipError_t launch_export(const StateDesc& d, double* dst, hipStream_t s);
hipError_t launch_import(const StateDesc& d, void* dst, const double* src, hipStream_t s);
// Writes out[0..4] = (sum Nu_local over the face or 0, KE, sum T, max|u|, #non-finite).
// `partials` must hold at least diag_partials_needed(...) doubles.
size_t diag_partials_needed(const StateDesc& d);
hipError_t launch_diagnostics(const StateDesc& d, int face, const FaceDev& fd, double dT_ref,
                              double* partials, double* out, hipStream_t s);

}  // namespace fpc
