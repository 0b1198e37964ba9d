// Adjoint stream-collide step and adjoint of the initial collision.
//
// One time step is S_n = Phi(S_{n-1}) = collide(pull(S_{n-1})) (see
// fpc_step.hip).  For an objective J whose direct dependence on S_n comes
// through the time-n macros (rho, u, T, recovered from S_n), the adjoint
// recursion lambda_{n-1} = Phi^T (lambda_n + dJ/dS_n) is evaluated per node x:
//   1. pull S_{n-1} at x exactly as the forward step (same wall rules),
//   2. redo the collision on plain populations, keeping the tape,
//   3. add the objective's seed on S_n(x) (weights on T_n(x) and/or the
//      kinetic energy 1/2 rho |u|^2), take lambda_n(x),
//   4. back-propagate through the collision (fpc_adjoint.h),
//   5. push each incoming link's adjoint to the slot it was pulled from:
//      the neighbour's slot (x - e_a, a) for streaming and periodic links, the
//      node's own opposite slot for wall links (sign +1 for bounce-back and
//      moving walls, -1 for the Dirichlet anti-bounce-back, whose wall
//      temperature receives 2 w^T_a = c^_s^2 times the link adjoint).
// Streaming plus the wall rules read every slot of S_{n-1} exactly once, so
// every slot of lambda_{n-1} is written exactly once: no atomics, and each
// wall-temperature gradient entry has a single owner thread per launch.
#include <type_traits>

#include "fpc_adjoint.h"
#include "fpc_gather.h"

// Extra attributes of the 3D FP32 adjoint step kernel: its natural register
// count sits just above the 168 VGPRs that allow 3 waves per SIMD.
#ifndef FPC_ADJ3F_ATTR
#define FPC_ADJ3F_ATTR __attribute__((amdgpu_waves_per_eu(3)))
#endif

namespace fpc {
namespace {

using namespace stream;

template <int D>
struct LinkOf {
  static constexpr int Qf = D == 2 ? kQ2 : kQ3;
  static constexpr int Qg = D == 2 ? kQ2T : kQ3T;
  static constexpr int ex(int a) { return D == 2 ? D2_EX[a] : D3_EX[a]; }
  static constexpr int ey(int a) { return D == 2 ? D2_EY[a] : D3_EY[a]; }
  static constexpr int ez(int a) { return D == 2 ? 0 : D3_EZ[a]; }
  static constexpr int opp(int a) { return D == 2 ? D2_OPP[a] : d3_opp(a); }
  static constexpr double w(int a) { return D == 2 ? w2(a) : w3(a); }
};

// Seed of the objective on S_n(x): weights on T_n(x) and on the kinetic energy.
template <class R, int D, int UP>
__device__ __forceinline__ void add_seed(const adj::Tape<R, D>& t, const CollParams<R>& c, double dJdT, double ke,
                                         R* fb, R* gb) {
  using Lk = LinkOf<D>;
  R gs = R(dJdT);
  if (ke != 0.0) {
    const R kw = R(ke);
    R u2 = R(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) u2 += t.u[ax] * t.u[ax];
#pragma unroll
    for (int q = 0; q < Lk::Qf; ++q) {
      R eu = R(Lk::ex(q)) * t.u[0] + R(Lk::ey(q)) * t.u[1];
      if (D == 3) eu += R(Lk::ez(q)) * t.u[2];
      fb[q] += kw * (R(-0.5) * u2 + eu);
    }
    gs += kw * (R(-0.5) * c.gbeta * t.u[UP]);
  }
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) gb[q] += gs;
}

template <class R>
struct AdjArgs {
  StepArgs<R> s;      // s.src = S_{n-1} (storage format); s.dst unused
  const R* lam_in;    // adjoint of S_n (same layout as the state)
  R* lam_out;         // adjoint of S_{n-1}
  const double* dJdT; // per-node seed on T_n, or null
  double ke;          // weight of the kinetic-energy seed
  double* dtheta[6];  // per-face wall-temperature gradient (accumulated), or null
};

// Adjoint of the streaming step for one node: push the adjoint of each
// incoming link to the slot it was read from (Edges: same classification as
// the gather).  Thermal Dirichlet links carry the factor -1 of the
// anti-bounce-back; their wall temperature receives 2 w^T_a = c^_s^2 times the
// link adjoint.
template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX>
struct Scatter {
  using E = Edges<L, R, CX, CY, CZ, PX>;
  const AdjArgs<R>& A;
  const M& m;
  E e;
  int x, y, z;

  __device__ __forceinline__ Scatter(const AdjArgs<R>& A_, const M& m_, int x_, int y_, int z_, unsigned node)
      : A(A_), m(m_), e(A_.s, x_, y_, z_, node), x(x_), y(y_), z(z_) {}

  template <int Q, int QBASE>
  __device__ __forceinline__ void push(R v) const {
    constexpr bool TH = QBASE != 0;
    constexpr int ex = lex<L, TH>(Q);
    if (!E::template checked<Q, TH>()) {
      m.store_tile(QBASE + Q, e.tl.template base<ex>(e.template dtile<Q, TH>()), e.tl.template lane<ex>(), v);
      return;
    }
    const long long sh = e.template shift<Q, TH>();
    bool wx = false, wy = false, wz = false;
    const unsigned idx = e.template source<Q, TH>(wx, wy, wz);
    if (E::template wrap_only<Q, TH>()) {
      m.store_at(QBASE + Q, sh, idx, v);
      return;
    }
    const bool wall = wx || wy || wz;
    R out = v;
    if (QBASE != 0 && Q != 0) {
      constexpr int ey = ley<L, TH>(Q), ez = lez<L, TH>(Q);
      constexpr int F = ex > 0 ? 0 : (ex < 0 ? 1 : (ey > 0 ? 2 : (ey < 0 ? 3 : (ez > 0 ? 4 : 5))));
      constexpr int k = F >> 1;
      const StepArgs<R>& a = A.s;
      if (wall && a.face[F].dirichlet) {
        out = -v;
        if (A.dtheta[F]) {
          const size_t t = k == 0 ? (size_t)z * a.ny + y : (k == 1 ? (size_t)z * a.nx + x : (size_t)y * a.nx + x);
          A.dtheta[F][t] += (double)(a.c.cs2T * v);
        }
      }
    }
    m.store_sel(wall, QBASE + lopp<L, TH>(Q), e.node, QBASE + Q, sh, idx, out);
  }
};

template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX = false>
__device__ __forceinline__ void scatter(const AdjArgs<R>& A, const M& mL, int x, int y, int z, unsigned node,
                                        const R (&fb)[L::Qf], const R (&gb)[L::Qg]) {
  const Scatter<L, R, M, CX, CY, CZ, PX> sc(A, mL, x, y, z, node);
  if constexpr (L::D == 2) {
    sc.template push<0, 0>(fb[0]); sc.template push<1, 0>(fb[1]); sc.template push<2, 0>(fb[2]);
    sc.template push<3, 0>(fb[3]); sc.template push<4, 0>(fb[4]); sc.template push<5, 0>(fb[5]);
    sc.template push<6, 0>(fb[6]); sc.template push<7, 0>(fb[7]); sc.template push<8, 0>(fb[8]);
    sc.template push<0, kQ2>(gb[0]); sc.template push<1, kQ2>(gb[1]); sc.template push<2, kQ2>(gb[2]);
    sc.template push<3, kQ2>(gb[3]); sc.template push<4, kQ2>(gb[4]);
  } else {
#define FPC_P(Q) sc.template push<Q, 0>(fb[Q]);
    FPC_P(0) FPC_P(1) FPC_P(2) FPC_P(3) FPC_P(4) FPC_P(5) FPC_P(6) FPC_P(7) FPC_P(8)
    FPC_P(9) FPC_P(10) FPC_P(11) FPC_P(12) FPC_P(13) FPC_P(14) FPC_P(15) FPC_P(16) FPC_P(17)
    FPC_P(18) FPC_P(19) FPC_P(20) FPC_P(21) FPC_P(22) FPC_P(23) FPC_P(24) FPC_P(25) FPC_P(26)
#undef FPC_P
    sc.template push<0, kQ3>(gb[0]); sc.template push<1, kQ3>(gb[1]); sc.template push<2, kQ3>(gb[2]);
    sc.template push<3, kQ3>(gb[3]); sc.template push<4, kQ3>(gb[4]); sc.template push<5, kQ3>(gb[5]);
    sc.template push<6, kQ3>(gb[6]);
  }
}

// M: addressing policy of S_{n-1} (read) and of the adjoint pair (lam_in
// read, lam_out written); Buf32 below 4 GiB per buffer, else Glob64.
// The edge variant is chosen per wavefront (ballot) for the gather and again
// for the scatter; the collision and its adjoint in between are shared.
template <class L, class R, class M, int UP, bool STD>
__device__ __forceinline__ void adjoint_step(const AdjArgs<R>& A, unsigned total_bytes) {
  constexpr int D = L::D;
  const StepArgs<R>& a = A.s;
  // XCD-aware block order in 2D as in the forward step (the 3D in-plane order
  // measured neutral for the adjoint)
  const dim3 bi = (D == 2 && FPC_XCD_2D) ? xcd_block() : dim3(blockIdx.x, blockIdx.y, blockIdx.z);
  const int x = bi.x * blockDim.x + threadIdx.x;
  const int y = bi.y * blockDim.y + threadIdx.y;
  const int z = bi.z;
  if (x >= a.nx || y >= a.ny) return;
  const M mS(a.src, nullptr, total_bytes);
  const M mL(A.lam_in, A.lam_out, total_bytes);
  const unsigned node = node_of(x, y, z, a.nxp, a.ny);
  // which axes have an edge node in this wavefront (wave-uniform)
  const bool needx = __any(x == 0 || x == a.nx - 1);
  const bool needyz = __any(y == 0 || y == a.ny - 1) || (D == 3 && __any(z == 0 || z == a.nz - 1));
  const int variant = needyz ? 3 : (!needx ? 0 : (a.per[0] ? 1 : 2));
  const R Tr = tref(a, x, y, z);
  R f[L::Qf], g[L::Qg];
  if (variant == 0)
    gather<L, R, M, false, false, false>(a, mS, x, y, z, node, Tr, f, g);
  else if (variant == 1)
    gather<L, R, M, true, false, false, true>(a, mS, x, y, z, node, Tr, f, g);
  else if (variant == 2)
    gather<L, R, M, true, false, false>(a, mS, x, y, z, node, Tr, f, g);
  else
    gather<L, R, M, true, true, D == 3>(a, mS, x, y, z, node, Tr, f, g);
  if constexpr (kDeviations<R>) {
    // plain populations: add this node's storage references
#pragma unroll
    for (int q = 0; q < L::Qf; ++q) f[q] += R(L::w(q)) * a.c.rho_r;
#pragma unroll
    for (int q = 0; q < L::Qg; ++q) g[q] += L::template wT<R>(q, a.c.cs2T) * Tr;
  }
  adj::Tape<R, D> t;
  adj::forward<R, D, UP, STD>(f, g, a.c, t);
  R fb[L::Qf], gb[L::Qg];
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) fb[q] = mL.load(q, 0, node);
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) gb[q] = mL.load(L::Qf + q, 0, node);
  const size_t cell = ((size_t)z * a.ny + y) * a.nx + x;  // index of the unpadded node fields
  add_seed<R, D, UP>(t, a.c, A.dJdT ? A.dJdT[cell] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP, STD>(t, a.c, fb, gb);
  if (variant == 0)
    scatter<L, R, M, false, false, false>(A, mL, x, y, z, node, fb, gb);
  else if (variant == 1)
    scatter<L, R, M, true, false, false, true>(A, mL, x, y, z, node, fb, gb);
  else if (variant == 2)
    scatter<L, R, M, true, false, false>(A, mL, x, y, z, node, fb, gb);
  else
    scatter<L, R, M, true, true, D == 3>(A, mL, x, y, z, node, fb, gb);
}

// STD: the standard rate set (fpc_kernels.h standard_rates), whose unit
// rates fold at compile time.
template <class L, class R, class M, int UP, bool STD>
__global__ void __launch_bounds__(256) adjoint_step_kernel(AdjArgs<R> A, unsigned total_bytes) {
  adjoint_step<L, R, M, UP, STD>(A, total_bytes);
}
template <class L, class M, int UP, bool STD>
__global__ void __launch_bounds__(256) FPC_ADJ3F_ATTR adjoint_step_kernel_3f(AdjArgs<float> A, unsigned total_bytes) {
  adjoint_step<L, float, M, UP, STD>(A, total_bytes);
}

template <class R>
struct AdjInitArgs {
  StepArgs<R> s;       // geometry and parameters
  const double* T_init;
  const R* lam0;       // adjoint of S_0
  const double* dJdT;  // seed on T_0, or null
  double ke;
  double* dTinit;      // output: dJ/dT_init per node
};

template <int D, class R, int UP>
__global__ void __launch_bounds__(256) adjoint_init_kernel(AdjInitArgs<R> A) {
  using Lk = LinkOf<D>;
  const StepArgs<R>& a = A.s;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  constexpr int Q = Lk::Qf + Lk::Qg;
  const size_t node = ((size_t)z * a.ny + y) * a.nx + x;  // unpadded node fields
  const unsigned n = node_of(x, y, z, a.nxp, a.ny);         // storage layout
  R f[Lk::Qf], g[Lk::Qg], wg[Lk::Qg];
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) f[q] = R(Lk::w(q)) * a.rho_w;
  const R Ti = R(A.T_init[node]);
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) {
    wg[q] = q == 0 ? R(1) - R(D) * a.c.cs2T : R(0.5) * a.c.cs2T;
    g[q] = wg[q] * Ti;
  }
  adj::Tape<R, D> t;
  adj::forward<R, D, UP>(f, g, a.c, t);
  R fb[Lk::Qf], gb[Lk::Qg];
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) fb[q] = A.lam0[elem64<Q>(q, n)];
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) gb[q] = A.lam0[elem64<Q>(Lk::Qf + q, n)];
  add_seed<R, D, UP>(t, a.c, A.dJdT ? A.dJdT[node] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP>(t, a.c, fb, gb);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) s += (double)(wg[q] * gb[q]);
  A.dTinit[node] = s;
}

template <int D, class R, int UP>
hipError_t launch_adj(const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  using L = typename std::conditional<D == 2, Lat2, Lat3>::type;
  const StepArgs<R>& a = step ? step->s : init->s;
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  const dim3 block(bx, by, 1);
  const dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (step) {
    constexpr int Q = L::Qf + L::Qg;
    const double bytes = (double)a.nxp * a.ny * a.nz * Q * sizeof(R);
    const bool std_rates = standard_rates(a, D, L::Qg);
    if constexpr (D == 3 && sizeof(R) == 4) {
      if (bytes < 4294967296.0) {
        if (std_rates)
          adjoint_step_kernel_3f<L, Buf32<R, Q>, UP, true><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
        else
          adjoint_step_kernel_3f<L, Buf32<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
      } else {
        adjoint_step_kernel_3f<L, Glob64<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, 0u);
      }
    } else {
      if (bytes < 4294967296.0) {
        if (std_rates)
          adjoint_step_kernel<L, R, Buf32<R, Q>, UP, true><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
        else
          adjoint_step_kernel<L, R, Buf32<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
      } else {
        adjoint_step_kernel<L, R, Glob64<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, 0u);
      }
    }
  } else {
    adjoint_init_kernel<D, R, UP><<<grid, block, 0, st>>>(*init);
  }
  return hipGetLastError();
}

template <class R>
hipError_t dispatch(int dim, int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  if (dim == 2) return up == 0 ? launch_adj<2, R, 0>(step, init, st) : launch_adj<2, R, 1>(step, init, st);
  if (up == 0) return launch_adj<3, R, 0>(step, init, st);
  if (up == 1) return launch_adj<3, R, 1>(step, init, st);
  return launch_adj<3, R, 2>(step, init, st);
}

}  // namespace

template <class R>
hipError_t launch_adjoint_step(const StepArgs<R>& a, int dim, int up, const void* lam_in, void* lam_out,
                               const double* dJdT, double ke, double* const dtheta[6], hipStream_t st) {
  AdjArgs<R> A;
  A.s = a;
  A.lam_in = static_cast<const R*>(lam_in);
  A.lam_out = static_cast<R*>(lam_out);
  A.dJdT = dJdT;
  A.ke = ke;
  for (int f = 0; f < 6; ++f) A.dtheta[f] = dtheta ? dtheta[f] : nullptr;
  return dispatch<R>(dim, up, &A, nullptr, st);
}

template <class R>
hipError_t launch_adjoint_init(const StepArgs<R>& a, int dim, int up, const double* T_init, const void* lam0,
                               const double* dJdT, double ke, double* dTinit, hipStream_t st) {
  AdjInitArgs<R> A;
  A.s = a;
  A.T_init = T_init;
  A.lam0 = static_cast<const R*>(lam0);
  A.dJdT = dJdT;
  A.ke = ke;
  A.dTinit = dTinit;
  return dispatch<R>(dim, up, nullptr, &A, st);
}

template hipError_t launch_adjoint_step<double>(const StepArgs<double>&, int, int, const void*, void*, const double*,
                                                double, double* const[6], hipStream_t);
template hipError_t launch_adjoint_step<float>(const StepArgs<float>&, int, int, const void*, void*, const double*,
                                               double, double* const[6], hipStream_t);
template hipError_t launch_adjoint_init<double>(const StepArgs<double>&, int, int, const double*, const void*,
                                                const double*, double, double*, hipStream_t);
template hipError_t launch_adjoint_init<float>(const StepArgs<float>&, int, int, const double*, const void*,
                                               const double*, double, double*, hipStream_t);

}  // namespace fpc
