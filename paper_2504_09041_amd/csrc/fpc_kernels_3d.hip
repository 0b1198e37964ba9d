// Fused pull-stream + collide kernel, D3Q27 fluid + D3Q7 thermal.
//
// Same structure as the 2D kernel: one thread per node pulls its 27 + 7
// incoming populations from S_{n-1} (or applies the halfway wall rules of
// Sec. 6.1 at its own node), collides in registers (collide3d) and stores its
// 34 values to S_n.  SoA planes [z][y][x]: a wavefront reads contiguous runs
// of one plane shifted by at most one element along x and by whole rows or
// layers along y and z.
#include "fpc_kernels.h"

namespace fpc {
namespace {

template <class R>
struct Pull3 {
  const StepArgs<R>& a;
  int x, y, z;
  size_t node;

  // Wall-side data of face F (compile-time index, so the argument block is
  // never indexed dynamically).
  template <int F>
  __device__ __forceinline__ R lid_term(int ex, int ey, int ez, double w) const {
    if (!a.face[F].lid) return R(0);
    const double eu = ex * a.face[F].uw[0] + ey * a.face[F].uw[1] + ez * a.face[F].uw[2];
    return R(2.0 * 3.0 * w) * a.rho_w * R(eu);
  }

  template <int F>
  __device__ __forceinline__ R dirichlet(R bb) const {
    if (!a.face[F].dirichlet) return bb;
    double Tw = a.face[F].Tw;
    if (a.face[F].Tprof) {
      constexpr int k = F >> 1;
      const size_t t = k == 0 ? (size_t)z * a.ny + y : (k == 1 ? (size_t)z * a.nx + x : (size_t)y * a.nx + x);
      Tw = a.face[F].Tprof[t];
    }
    return -bb + a.c.cs2T * (R(Tw) - a.c.T_r);  // 2 w^T_a = c^_s^2 on axis links
  }

  template <int A>
  __device__ __forceinline__ R f() const {
    constexpr int ex = D3_EX[A], ey = D3_EY[A], ez = D3_EZ[A];
    constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3, FZ = ez > 0 ? 4 : 5;
    int xs = x - ex, ys = y - ey, zs = z - ez;
    bool cx = false, cy = false, cz = false;
    if (ex != 0 && (xs < 0 || xs >= a.nx)) {
      if (a.per[0]) xs = xs < 0 ? a.nx - 1 : 0;
      else cx = true;
    }
    if (ey != 0 && (ys < 0 || ys >= a.ny)) {
      if (a.per[1]) ys = ys < 0 ? a.ny - 1 : 0;
      else cy = true;
    }
    if (ez != 0 && (zs < 0 || zs >= a.nz)) {
      if (a.per[2]) zs = zs < 0 ? a.nz - 1 : 0;
      else cz = true;
    }
    const int nc = (int)cx + (int)cy + (int)cz;
    if (nc == 0) return a.src[A * a.plane + ((size_t)zs * a.ny + ys) * a.nx + xs];
    R v = a.src[(size_t)d3_opp(A) * a.plane + node];
    if (nc == 1) {
      if (cx) v += lid_term<FX>(ex, ey, ez, w3(A));
      else if (cy) v += lid_term<FY>(ex, ey, ez, w3(A));
      else v += lid_term<FZ>(ex, ey, ez, w3(A));
    }
    return v;
  }

  // Thermal D3Q7 link A (axis links only: at most one face can be crossed).
  template <int A>
  __device__ __forceinline__ R g() const {
    constexpr int ex = D3_EX[A], ey = D3_EY[A], ez = D3_EZ[A];
    constexpr size_t base = kQ3;
    constexpr int F = ex > 0 ? 0 : (ex < 0 ? 1 : (ey > 0 ? 2 : (ey < 0 ? 3 : (ez > 0 ? 4 : 5))));
    constexpr int k = F >> 1;
    if (A == 0) return a.src[base * a.plane + node];
    const int c = k == 0 ? x : (k == 1 ? y : z);
    const int n = k == 0 ? a.nx : (k == 1 ? a.ny : a.nz);
    const int e = k == 0 ? ex : (k == 1 ? ey : ez);
    int cs = c - e;
    bool wall = false;
    if (cs < 0 || cs >= n) {
      if (a.per[k]) cs = cs < 0 ? n - 1 : 0;
      else wall = true;
    }
    if (wall) return dirichlet<F>(a.src[(base + d3_opp(A)) * a.plane + node]);
    const int xs = k == 0 ? cs : x, ys = k == 1 ? cs : y, zs = k == 2 ? cs : z;
    return a.src[(base + A) * a.plane + ((size_t)zs * a.ny + ys) * a.nx + xs];
  }
};

template <class R, int UP, int MODE>
__global__ void __launch_bounds__(256) step3d_kernel(StepArgs<R> a, const double* __restrict__ T_init) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const size_t node = ((size_t)z * a.ny + y) * a.nx + x;
  R f[kQ3], g[kQ3T];
  if (MODE == 0) {
    const Pull3<R> p{a, x, y, z, node};
#define FPC_PULLF(A) f[A] = p.template f<A>();
    FPC_PULLF(0) FPC_PULLF(1) FPC_PULLF(2) FPC_PULLF(3) FPC_PULLF(4) FPC_PULLF(5) FPC_PULLF(6)
    FPC_PULLF(7) FPC_PULLF(8) FPC_PULLF(9) FPC_PULLF(10) FPC_PULLF(11) FPC_PULLF(12) FPC_PULLF(13)
    FPC_PULLF(14) FPC_PULLF(15) FPC_PULLF(16) FPC_PULLF(17) FPC_PULLF(18) FPC_PULLF(19) FPC_PULLF(20)
    FPC_PULLF(21) FPC_PULLF(22) FPC_PULLF(23) FPC_PULLF(24) FPC_PULLF(25) FPC_PULLF(26)
#undef FPC_PULLF
    g[0] = p.template g<0>(); g[1] = p.template g<1>(); g[2] = p.template g<2>();
    g[3] = p.template g<3>(); g[4] = p.template g<4>(); g[5] = p.template g<5>();
    g[6] = p.template g<6>();
  } else {
    const R drw = a.rho_w - a.c.rho_r;
#pragma unroll
    for (int q = 0; q < kQ3; ++q) f[q] = R(w3(q)) * drw;
    const R dT = R(T_init[node]) - a.c.T_r;
    const R wa = R(0.5) * a.c.cs2T;
    g[0] = (R(1) - R(3) * a.c.cs2T) * dT;
#pragma unroll
    for (int q = 1; q < kQ3T; ++q) g[q] = wa * dT;
  }
  collide3d<R, UP>(f, g, a.c, (Macros<R>*)nullptr);
#pragma unroll
  for (int q = 0; q < kQ3; ++q) a.dst[q * a.plane + node] = f[q];
#pragma unroll
  for (int q = 0; q < kQ3T; ++q) a.dst[(kQ3 + q) * a.plane + node] = g[q];
}

template <class R, int UP>
hipError_t launch_up(const StepArgs<R>& a, const double* T_init, int mode, hipStream_t s) {
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  dim3 block(bx, by, 1);
  dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (mode == 0)
    step3d_kernel<R, UP, 0><<<grid, block, 0, s>>>(a, T_init);
  else
    step3d_kernel<R, UP, 1><<<grid, block, 0, s>>>(a, T_init);
  return hipGetLastError();
}

}  // namespace

template <class R>
hipError_t launch_step3d(const StepArgs<R>& a, int up, const double* T_init, int mode, hipStream_t s) {
  switch (up) {
    case 0: return launch_up<R, 0>(a, T_init, mode, s);
    case 1: return launch_up<R, 1>(a, T_init, mode, s);
    default: return launch_up<R, 2>(a, T_init, mode, s);
  }
}

template hipError_t launch_step3d<double>(const StepArgs<double>&, int, const double*, int, hipStream_t);
template hipError_t launch_step3d<float>(const StepArgs<float>&, int, const double*, int, hipStream_t);

}  // namespace fpc
