// Fused pull-stream + collide kernel, D2Q9 fluid + D2Q5 thermal.
//
// One thread per node.  Each thread pulls its 9 + 5 incoming populations
// f_a(x) = f~_a(x - e_a) from S_{n-1} (Eq. LBMsteps-stream, LBMsteps-streamg)
// or, when x - e_a lies outside a wall face, applies the halfway wall rule at
// its own node (Sec. 6.1): bounce-back f_a = f~_abar, moving wall
// f_a = f~_abar + 2 w_a rho_w (e_a . u_w) / c_s^2, adiabatic g_a = g~_abar,
// Dirichlet g_a = -g~_abar + 2 w^T_a T_w; then collides in registers and
// stores its own 14 values to S_n.  Storage is SoA: plane q holds N values
// [y][x], so the loads of a wavefront are contiguous runs shifted by at most
// one element and the stores are fully coalesced.
#include "fpc_kernels.h"

namespace fpc {
namespace {

template <class R>
struct Pull2 {
  const StepArgs<R>& a;
  int x, y;
  size_t node;

  // Wall-side data of face F (compile-time index, so the argument block is
  // never indexed dynamically).
  template <int F>
  __device__ __forceinline__ R lid_term(int ex, int ey, double w) const {
    if (!a.face[F].lid) return R(0);
    const double eu = ex * a.face[F].uw[0] + ey * a.face[F].uw[1];
    return R(2.0 * 3.0 * w) * a.rho_w * R(eu);
  }

  template <int F>
  __device__ __forceinline__ R dirichlet(R bb) const {
    if (!a.face[F].dirichlet) return bb;
    const double Tw = a.face[F].Tprof ? a.face[F].Tprof[F < 2 ? y : x] : a.face[F].Tw;
    return -bb + a.c.cs2T * (R(Tw) - a.c.T_r);  // 2 w^T_a = c^_s^2 on axis links
  }

  // Incoming fluid population of link A.
  template <int A>
  __device__ __forceinline__ R f() const {
    constexpr int ex = D2_EX[A], ey = D2_EY[A];
    constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3;
    int xs = x - ex, ys = y - ey;
    bool cx = false, cy = false;
    if (ex != 0 && (xs < 0 || xs >= a.nx)) {
      if (a.per[0]) xs = xs < 0 ? a.nx - 1 : 0;
      else cx = true;
    }
    if (ey != 0 && (ys < 0 || ys >= a.ny)) {
      if (a.per[1]) ys = ys < 0 ? a.ny - 1 : 0;
      else cy = true;
    }
    if (!cx && !cy) return a.src[A * a.plane + (size_t)ys * a.nx + xs];
    R v = a.src[D2_OPP[A] * a.plane + node];
    if (cx != cy) v += cx ? lid_term<FX>(ex, ey, w2(A)) : lid_term<FY>(ex, ey, w2(A));
    return v;
  }

  // Incoming thermal population of D2Q5 link A (0..4; axis links).
  template <int A>
  __device__ __forceinline__ R g() const {
    constexpr int ex = D2_EX[A], ey = D2_EY[A];
    constexpr size_t base = kQ2;
    constexpr int F = ex > 0 ? 0 : (ex < 0 ? 1 : (ey > 0 ? 2 : 3));
    if (A == 0) return a.src[base * a.plane + node];
    int xs = x - ex, ys = y - ey;
    bool wall = false;
    if (ex != 0 && (xs < 0 || xs >= a.nx)) {
      if (a.per[0]) xs = xs < 0 ? a.nx - 1 : 0;
      else wall = true;
    }
    if (ey != 0 && (ys < 0 || ys >= a.ny)) {
      if (a.per[1]) ys = ys < 0 ? a.ny - 1 : 0;
      else wall = true;
    }
    if (wall) return dirichlet<F>(a.src[(base + D2_OPP[A]) * a.plane + node]);
    return a.src[(base + A) * a.plane + (size_t)ys * a.nx + xs];
  }
};

template <class R, int UP, int MODE>
__global__ void __launch_bounds__(256) step2d_kernel(StepArgs<R> a, const double* __restrict__ T_init) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const size_t node = (size_t)y * a.nx + x;
  R f[kQ2], g[kQ2T];
  if (MODE == 0) {
    const Pull2<R> p{a, x, y, node};
    f[0] = p.template f<0>(); f[1] = p.template f<1>(); f[2] = p.template f<2>();
    f[3] = p.template f<3>(); f[4] = p.template f<4>(); f[5] = p.template f<5>();
    f[6] = p.template f<6>(); f[7] = p.template f<7>(); f[8] = p.template f<8>();
    g[0] = p.template g<0>(); g[1] = p.template g<1>(); g[2] = p.template g<2>();
    g[3] = p.template g<3>(); g[4] = p.template g<4>();
  } else {
    // initial pre-collision state: f = w rho_w, g = w^T T_init (stored minus offsets)
    const R drw = a.rho_w - a.c.rho_r;
#pragma unroll
    for (int q = 0; q < kQ2; ++q) f[q] = R(w2(q)) * drw;
    const R dT = R(T_init[node]) - a.c.T_r;
    const R wa = R(0.5) * a.c.cs2T;
    g[0] = (R(1) - R(2) * a.c.cs2T) * dT;
    g[1] = g[2] = g[3] = g[4] = wa * dT;
  }
  collide2d<R, UP>(f, g, a.c, (Macros<R>*)nullptr);
#pragma unroll
  for (int q = 0; q < kQ2; ++q) a.dst[q * a.plane + node] = f[q];
#pragma unroll
  for (int q = 0; q < kQ2T; ++q) a.dst[(kQ2 + q) * a.plane + node] = g[q];
}

template <class R, int UP>
hipError_t launch_up(const StepArgs<R>& a, const double* T_init, int mode, hipStream_t s) {
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  dim3 block(bx, by, 1);
  dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, 1);
  if (mode == 0)
    step2d_kernel<R, UP, 0><<<grid, block, 0, s>>>(a, T_init);
  else
    step2d_kernel<R, UP, 1><<<grid, block, 0, s>>>(a, T_init);
  return hipGetLastError();
}

}  // namespace

template <class R>
hipError_t launch_step2d(const StepArgs<R>& a, int up, const double* T_init, int mode, hipStream_t s) {
  return up == 0 ? launch_up<R, 0>(a, T_init, mode, s) : launch_up<R, 1>(a, T_init, mode, s);
}

template hipError_t launch_step2d<double>(const StepArgs<double>&, int, const double*, int, hipStream_t);
template hipError_t launch_step2d<float>(const StepArgs<float>&, int, const double*, int, hipStream_t);

}  // namespace fpc
