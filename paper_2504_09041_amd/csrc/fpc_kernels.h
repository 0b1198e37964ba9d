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

// Wall-Nusselt accumulation fused into the step (off when slot is NULL):
// every node of the two layers next to `face` adds its share of
// weight * <Nu>_face of the new time level (Sec. 6.1 stencil), summed per
// wavefront into slot[] (one slot per 64-node tile of those layers, written
// only by that tile's wavefront, so the per-slot sums over the steps of a run
// are deterministic).
struct NuAcc {
  double* slot;
  int face;
  int nk;              // nodes along the face normal (L)
  int nt;              // nodes along the faster tangential axis (profile row length)
  int ns;              // nodes along the slower tangential axis
  double scale;        // -(L / dT_ref) * weight / (nodes on the face)
  double Tw;           // uniform wall temperature
  const double* Tprof; // optional per-node wall temperature (profile layout)
  double T_o, Tg[3];   // thermal storage reference in FP64 (zero for FP64 storage)
};

// Diagnostics fused into a step (off when part is NULL): after its stores,
// every wavefront reduces, over its tile, the per-node FP64 values of the
// diagnostics (kinetic energy 1/2 rho |u|^2, T, |u|, non-finite flag) formed
// from the stored post-collision values exactly as fpc_diagnostics forms them,
// and writes the four results to part[4 tile + k]; a fixed-order reduction
// over the tiles follows the step.
struct DiagAcc {
  double* part;
  double rho_r;         // storage offset of f (0 for FP64 storage)
  double T_o, Tg[3];    // thermal storage reference in FP64 (zero for FP64 storage)
  double gbeta, T0;     // buoyancy (F = gbeta (T - T0) along the up axis)
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
  NuAcc obj;
  DiagAcc dg;
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

// Whether the rates form the standard set of rate_f / rate_g: the viscous
// slots share one rate, the thermal first-order slots share one rate, and
// every other slot in use relaxes at exactly 1.  Kernels built for that set
// (STD = true) take those rates as compile-time constants, and with them the
// FP attractors and (on the paper's D2Q9 / D3Q15 thermal lattices, the only
// ones where it differs) thermal option A.
template <class R>
inline bool standard_rates(const StepArgs<R>& a, int D, int Qg) {
  if (a.c.model != 0) return false;
  if (a.c.topt != 0 && Qg != (D == 2 ? 5 : 7)) return false;
  const int Qf = D == 2 ? kQ2 : kQ3;
  for (int k = 1; k < Qf; ++k) {
    const bool nu = D == 2 ? (k == 4 || k == 5) : (k == 4 || k == 5 || k == 6 || k == 8 || k == 9);
    if (nu ? a.c.om[k] != a.c.om[4] : a.c.om[k] != R(1)) return false;
  }
  for (int k = 1; k < Qg; ++k) {
    const bool first = k <= D;
    if (first ? a.c.omg[k] != a.c.omg[1] : a.c.omg[k] != R(1)) return false;
  }
  return true;
}

// Launchers of the fused step (defined in fpc_step.hip).
// tk: thermal lattice, 0 = D2Q5 / D3Q7, 1 = D2Q9 / D3Q15.
// mode: 0 = step (pull from args.src), 1 = init (equilibrium from T_init).
template <class R>
hipError_t launch_step2d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s);
template <class R>
hipError_t launch_step3d(const StepArgs<R>& a, int up, int tk, const double* T_init, int mode, hipStream_t s);

// Several steps in one cooperative launch (small grids, every lattice pair in
// 2D and in 3D FP32, standard rate set, state below the non-temporal
// threshold): see
// step_multi_kernel in fpc_step.hip.  The host fills everything but nwork,
// which the launcher sets.
struct MultiCtl {
  unsigned* bar;        // full barrier's word (zero between launches)
  int* err;             // sticky: a barrier wait ran out
  unsigned* place;      // two XCD-placement words, used by alternate launches
  unsigned* arrive;     // light barrier: one arrival word per working block
  unsigned* release;    // light barrier: release word
  unsigned spin_limit;  // polls before giving up
  unsigned nwork;       // working blocks (the launch has nwork * kXcds), at most 64
  int nsteps;
  int seq;              // launch number (selects the placement word)
  unsigned gen;         // light-barrier number of this launch's first step (unique per launch)
};
// Working blocks of 256 threads (64, 128 or 256 along x) that cover the grid.
inline unsigned multi_work_blocks(int nx, int ny, int nz) {
  const int bx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  return (unsigned)((nx + bx - 1) / bx) * (unsigned)((ny + by - 1) / by) * (unsigned)nz;
}
template <class R>
hipError_t launch_step_multi(const StepArgs<R>& a, int dim, int up, int tk, const MultiCtl& c, hipStream_t s);

// Adjoint kernels (fpc_adjoint.hip).  `a.src` is S_{n-1} (adjoint step) or
// unused (adjoint of the initial collision).  tk: thermal lattice, 0 = D2Q5 /
// D3Q7, 1 = the paper's D2Q9 / D3Q15.
template <class R>
hipError_t launch_adjoint_step(const StepArgs<R>& a, int dim, int up, int tk, const void* lam_in, void* lam_out,
                               const double* dJdT, double ke, double* const dtheta[6], hipStream_t s);
template <class R>
hipError_t launch_adjoint_init(const StepArgs<R>& a, int dim, int up, int tk, const double* T_init, const void* lam0,
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
// Diagnostics reductions.  Writes out[0..4] = (mean Nu over the face or 0,
// KE, sum T, max|u|, number of non-finite nodes) with a fixed summation order
// for a given grid.  `scratch` (device) must hold kDiagScratchDoubles doubles;
// `out` (device, 5 doubles) must not overlap the first kDiagNodeBlocks * 4 +
// kDiagFaceBlocks of them.
constexpr unsigned kDiagNodeBlocks = 1024;  // stage-1 blocks over the nodes (at most)
constexpr unsigned kDiagFaceBlocks = 64;    // stage-1 blocks over a face (at most)
constexpr size_t kDiagScratchDoubles = (size_t)kDiagNodeBlocks * 4 + kDiagFaceBlocks + 8;
hipError_t launch_diagnostics(const StateDesc& d, int face, const FaceDev& fd, double dT_ref,
                              double* scratch, double* out, hipStream_t s);

// Local Nusselt number of every node of `face` (profile layout of
// fpc_params.wall_T_profile) into out.
hipError_t launch_nu_local(const StateDesc& d, int face, const FaceDev& fd, double dT_ref, double* out,
                           hipStream_t s);

// Slots of the fused wall-Nusselt accumulation for `face` (see NuAcc): one per
// tile of the two wall layers.  nu_slot_count is the number a face needs.
size_t nu_slot_count(int nx, int ny, int nz, int nxp, int face);
// acc[0] += sum of slot[0..count) in a fixed order (two stages, at most
// kDiagFaceBlocks blocks, partials in scratch[kDiagNodeBlocks * 4 ...]); the
// slots are zeroed.
hipError_t launch_nu_slots_reduce(double* slot, size_t count, double* scratch, double* acc, hipStream_t s);
// slot[0..count) = 0.
hipError_t launch_fill_zero(double* p, size_t count, hipStream_t s);
// Reduction of the per-tile partials of a step with fused diagnostics
// (DiagAcc) in a fixed order: out[0] = the sum of the wall-Nusselt slots
// slot[0..nslots) (which are zeroed), or 0 when slot is NULL; out[1..4] =
// (KE, sum T, max |u|, non-finite nodes).  scratch: kDiagNodeBlocks * 4 +
// kDiagFaceBlocks doubles, not overlapping out.
hipError_t launch_diag_tiles(const double* part, size_t ntiles, double* slot, size_t nslots, double* scratch,
                             double* out, hipStream_t s);
// Seeds of the adjoint of J = weight * <Nu>_face (Sec. 6.1 stencil):
// dJdT[node] (N values, zero off the two wall layers) and, if dJdTw is not
// NULL, dJdTw[i] = dJ / dT_w at wall node i (profile layout).
hipError_t launch_nu_seed(const StateDesc& d, int face, double dT_ref, double weight, double* dJdT, double* dJdTw,
                          hipStream_t s);

}  // namespace fpc
