// Adjoint stream-collide step and adjoint of the initial collision.
//
// One time step is S_n = Phi(S_{n-1}) = collide(pull(S_{n-1})) (see
// fpc_step.hip).  The adjoint is carried between steps as mu_{n-1}, the
// adjoint of the pulled (pre-collision) populations that enter the collision
// of step n; the adjoint of the stored state S_{n-1} is lambda_{n-1} =
// pull^T mu_{n-1}.  For an objective J whose direct dependence on S_n comes
// through the time-n macros (rho, u, T, recovered from S_n), one adjoint step
//   mu_{n-1} = collide_n^T (pull^T mu_n + dJ/dS_n)
// is evaluated per node x:
//   1. pull S_{n-1} at x exactly as the forward step (same wall rules),
//   2. redo the collision on plain populations, keeping the tape,
//   3. form lambda_n(x) = (pull^T mu_n)(x): the transpose of the pull is a
//      pull in the opposite direction (Rev in fpc_gather.h): slot (x, a)
//      feeds the incoming link (x + e_a, a), or across a wall face the node's
//      own link (x, abar), with the factor -1 of the Dirichlet rule,
//   4. add the objective's seed on S_n(x) (weights on T_n(x) and/or the
//      kinetic energy 1/2 rho |u|^2),
//   5. back-propagate through the collision (fpc_adjoint.h): mu_{n-1}(x),
//      stored in x's own tile, and the Dirichlet wall temperature of each of
//      x's own Dirichlet links receives 2 w^T_a times its adjoint (see
//      theta_link).
// Every access of a node is a run of its own tile (stores) or a pulled run
// (loads), as in the forward step; each wall-temperature gradient entry has a
// single owner thread per launch.
//
// The kernels and their launch for one lattice pair (launch_adj); each
// lattice pair is instantiated in a source file of its own (fpc_adjoint.hip:
// D2Q9 + D2Q5; fpc_adjoint_d3q7.hip; fpc_adjoint_d2q9.hip and
// fpc_adjoint_d3q15.hip: the paper's thermal lattices), so that they compile
// in parallel.
#pragma once

#include <type_traits>
#include <utility>

#include "fpc_adjoint.h"
#include "fpc_gather.h"

namespace fpc {
namespace adjk {

using namespace stream;

// Seed of the objective on S_n(x): weights on T_n(x) and on the kinetic energy.
template <class L, class R, int UP>
__device__ __forceinline__ void add_seed(const adj::Tape<R, L::D, L::Qg>& t, const CollParams<R>& c, double dJdT,
                                         double ke, R* fb, R* gb) {
  constexpr int D = L::D;
  using Lk = L;
  R gs = R(dJdT);
  if (ke != 0.0) {
    const R kw = R(ke);
    R u2 = R(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) u2 += t.u[ax] * t.u[ax];
    const R base = R(-0.5) * u2;
#pragma unroll
    for (int q = 0; q < Lk::Qf; ++q) {
      // base + e_q . u over the non-zero components of e_q
      R v = base;
      if (Lk::ex(q) != 0) v = Lk::ex(q) > 0 ? v + t.u[0] : v - t.u[0];
      if (Lk::ey(q) != 0) v = Lk::ey(q) > 0 ? v + t.u[1] : v - t.u[1];
      if (D == 3 && Lk::ez(q) != 0) v = Lk::ez(q) > 0 ? v + t.u[2] : v - t.u[2];
      fb[q] += kw * v;
    }
    gs += kw * (R(-0.5) * c.gbeta * t.u[UP]);
  }
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) gb[q] += gs;
}

template <class R>
struct AdjArgs {
  StepArgs<R> s;      // s.src = S_{n-1} (storage format); s.dst unused
  const R* lam_in;    // mu_n: adjoint of the pulled populations of step n + 1 (state layout)
  R* lam_out;         // mu_{n-1}: the same for step n
  const double* dJdT; // per-node seed on T_n, or null
  double ke;          // weight of the kinetic-energy seed
  double* dtheta[6];  // per-face wall-temperature gradient (accumulated), or null
};

// lambda_n(x) = (pull^T mu_n)(x): the pull on the reversed lattice, with the
// factor -1 on thermal links whose x + e_a lies beyond a Dirichlet face.
template <class P, class R, size_t... I>
__device__ __forceinline__ void tpull_f(const P& p, R* fb, std::index_sequence<I...>) {
  bool wx, wy, wz;
  ((wx = wy = wz = false, fb[I] = p.template pull<(int)I, false>(wx, wy, wz)), ...);
}
template <class RL, int A, class P, class R>
__device__ __forceinline__ R tpull_g1(const P& p, const StepArgs<R>& a) {
  bool wx = false, wy = false, wz = false;
  const R v = p.template pull<A, true>(wx, wy, wz);
  if (A == 0 || !P::E::template checked<A, true>()) return v;
  constexpr int ex = RL::tex(A), ey = RL::tey(A), ez = RL::tez(A);
  constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3, FZ = ez > 0 ? 4 : 5;
  const bool dir = (ex != 0 && wx && a.face[FX].dirichlet) || (ey != 0 && wy && a.face[FY].dirichlet) ||
                   (ez != 0 && wz && a.face[FZ].dirichlet);
  return dir ? -v : v;
}
template <class RL, class P, class R, size_t... I>
__device__ __forceinline__ void tpull_g(const P& p, const StepArgs<R>& a, R* gb, std::index_sequence<I...>) {
  ((gb[I] = tpull_g1<RL, (int)I>(p, a)), ...);
}
template <class L, class R, class M, bool CX, bool CY, bool CZ, bool PX = false>
__device__ __forceinline__ void tgather(const StepArgs<R>& a, const M& m, int x, int y, int z, unsigned node,
                                        R (&fb)[L::Qf], R (&gb)[L::Qg]) {
  using RL = Rev<L>;
  const Gather<RL, R, M, CX, CY, CZ, PX> p(a, m, x, y, z, node, R(0));
  tpull_f(p, fb, std::make_index_sequence<L::Qf>{});
  tpull_g<RL>(p, a, gb, std::make_index_sequence<L::Qg>{});
}

// Wall-temperature gradient: each thermal link of x that met a Dirichlet face
// in the forward pull (g_a = -g~_abar + 2 w^T_a T_w, T_w the mean over the
// nd Dirichlet faces the link crosses: one for an axis link, up to two for a
// diagonal link of D2Q9 at an edge) adds 2 w^T_a / nd times its adjoint
// mu(x, a) to the entry of x on each of those faces (2 w^T_a = c^_s^2 on the
// axis links of D2Q5 / D3Q7).
template <class L, class R, int F>
__device__ __forceinline__ void theta_face(const AdjArgs<R>& AA, int x, int y, int z, R v) {
  constexpr int k = F >> 1;
  const StepArgs<R>& a = AA.s;
  if (AA.dtheta[F]) {
    const size_t t = k == 0 ? (size_t)z * a.ny + y : (k == 1 ? (size_t)z * a.nx + x : (size_t)y * a.nx + x);
    AA.dtheta[F][t] += (double)v;
  }
}
template <class L, class R, bool CX, bool CY, bool CZ, bool PX, int A>
__device__ __forceinline__ void theta_link(const AdjArgs<R>& AA, const Edges<L, R, CX, CY, CZ, PX>& e, int x, int y,
                                           int z, R v) {
  if constexpr (A == 0 || !Edges<L, R, CX, CY, CZ, PX>::template checked<A, true>()) {
    return;
  } else {
    const StepArgs<R>& a = AA.s;
    bool wx = false, wy = false, wz = false;
    (void)e.template source<A, true>(wx, wy, wz);
    constexpr int ex = L::tex(A), ey = L::tey(A), ez = L::tez(A);
    constexpr int FX = ex > 0 ? 0 : 1, FY = ey > 0 ? 2 : 3, FZ = ez > 0 ? 4 : 5;
    constexpr int nax = (ex != 0) + (ey != 0) + (ez != 0);
    const bool dx = ex != 0 && wx && a.face[FX].dirichlet;
    const bool dy = ey != 0 && wy && a.face[FY].dirichlet;
    const bool dz = ez != 0 && wz && a.face[FZ].dirichlet;
    const int nd = (int)dx + (int)dy + (int)dz;
    if (nd == 0) return;
    R s = R(2) * L::template wT<R>(A, a.c.cs2T) * v;
    if (nax > 1 && nd > 1) s = s / R(nd);
    if (ex != 0 && dx) theta_face<L, R, FX>(AA, x, y, z, s);
    if (ey != 0 && dy) theta_face<L, R, FY>(AA, x, y, z, s);
    if (ez != 0 && dz) theta_face<L, R, FZ>(AA, x, y, z, s);
  }
}
template <class L, class R, bool CX, bool CY, bool CZ, bool PX, size_t... I>
__device__ __forceinline__ void theta_links(const AdjArgs<R>& AA, int x, int y, int z, unsigned node, const R* gb,
                                            std::index_sequence<I...>) {
  if (!(CX || CY || CZ)) return;
  const Edges<L, R, CX, CY, CZ, PX> e(AA.s, x, y, z, node);
  (theta_link<L, R, CX, CY, CZ, PX, (int)I>(AA, e, x, y, z, gb[I]), ...);
}

// M: addressing policy of S_{n-1} (read) and of the adjoint pair (mu_n
// read, mu_{n-1} written); Buf32 below 4 GiB per buffer, else Glob64.  The
// edge variant is chosen per wavefront (ballot) for the forward pull, again
// for the transposed pull of mu_n and for the wall-temperature gradient; the
// collision and its adjoint in between, and the stores, are shared.
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
  adj::Tape<R, D, L::Qg> t;
  adj::forward<R, D, UP, STD, L::Qg>(f, g, a.c, t);
  R fb[L::Qf], gb[L::Qg];
  if (variant == 0)
    tgather<L, R, M, false, false, false>(a, mL, x, y, z, node, fb, gb);
  else if (variant == 1)
    tgather<L, R, M, true, false, false, true>(a, mL, x, y, z, node, fb, gb);
  else if (variant == 2)
    tgather<L, R, M, true, false, false>(a, mL, x, y, z, node, fb, gb);
  else
    tgather<L, R, M, true, true, D == 3>(a, mL, x, y, z, node, fb, gb);
  const size_t cell = ((size_t)z * a.ny + y) * a.nx + x;  // index of the unpadded node fields
  add_seed<L, R, UP>(t, a.c, A.dJdT ? A.dJdT[cell] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP, STD, L::Qg>(t, a.c, fb, gb);
  auto cur = mL.cursor(node);
#pragma unroll
  for (int q = 0; q < L::Qf; ++q) mL.template store_next<false>(cur, fb[q]);
#pragma unroll
  for (int q = 0; q < L::Qg; ++q) mL.template store_next<false>(cur, gb[q]);
  if (variant == 0) return;  // no wall links
  constexpr auto qg = std::make_index_sequence<L::Qg>{};
  if (variant == 1)
    theta_links<L, R, true, false, false, true>(A, x, y, z, node, gb, qg);
  else if (variant == 2)
    theta_links<L, R, true, false, false, false>(A, x, y, z, node, gb, qg);
  else
    theta_links<L, R, true, true, D == 3, false>(A, x, y, z, node, gb, qg);
}

// STD: the standard rate set (fpc_kernels.h standard_rates), whose unit
// rates fold at compile time.
template <class L, class R, class M, int UP, bool STD>
__global__ void __launch_bounds__(256) adjoint_step_kernel(AdjArgs<R> A, unsigned total_bytes) {
  adjoint_step<L, R, M, UP, STD>(A, total_bytes);
}
// Waves per SIMD that the 3D FP32 adjoint kernel of a lattice pair asks the
// register allocator to keep room for (1: no constraint).  The D3Q27 + D3Q15
// kernel holds 132 VGPRs at three waves; held to four it fits 128 VGPRs
// without spills and runs 4% faster at 128^3.  The D3Q27 + D3Q7 kernel fits
// four waves by itself (113 VGPRs).
template <class L>
struct Adj3fWaves {
  static constexpr unsigned value = 1;
};
template <>
struct Adj3fWaves<Lat3T15> {
  static constexpr unsigned value = 4;
};

template <class L, class M, int UP, bool STD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Adj3fWaves<L>::value)))
adjoint_step_kernel_3f(AdjArgs<float> A, unsigned total_bytes) {
  adjoint_step<L, float, M, UP, STD>(A, total_bytes);
}

template <class R>
struct AdjInitArgs {
  StepArgs<R> s;       // geometry and parameters
  const double* T_init;
  const R* lam0;       // mu_0: adjoint of the pulled populations of step 1
  const double* dJdT;  // seed on T_0, or null
  double ke;
  double* dTinit;      // output: dJ/dT_init per node
};

// lambda_0 = pull^T mu_0 (mu_0: the adjoint of the pulled populations of step
// 1), then the adjoint of the initial collision.  Blocks are whole multiples
// of 64 along x, so a wavefront owns one tile as in the step kernels.
template <class L, class R, int UP>
__global__ void __launch_bounds__(256) adjoint_init_kernel(AdjInitArgs<R> A) {
  constexpr int D = L::D;
  using Lk = L;
  const StepArgs<R>& a = A.s;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  constexpr int Q = Lk::Qf + Lk::Qg;
  const size_t node = ((size_t)z * a.ny + y) * a.nx + x;  // unpadded node fields
  const unsigned n = node_of(x, y, z, a.nxp, a.ny);         // storage layout
  const bool needx = __any(x == 0 || x == a.nx - 1);
  const bool needyz = __any(y == 0 || y == a.ny - 1) || (D == 3 && __any(z == 0 || z == a.nz - 1));
  R f[Lk::Qf], g[Lk::Qg], wg[Lk::Qg];
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) f[q] = R(Lk::w(q)) * a.rho_w;
  const R Ti = R(A.T_init[node]);
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) {
    wg[q] = L::template wT<R>(q, a.c.cs2T);
    g[q] = wg[q] * Ti;
  }
  adj::Tape<R, D, L::Qg> t;
  adj::forward<R, D, UP, false, L::Qg>(f, g, a.c, t);
  R fb[Lk::Qf], gb[Lk::Qg];
  using M = Glob64<R, Q>;
  const M m(A.lam0, nullptr, 0u);
  if (!needyz) {
    if (!needx)
      tgather<L, R, M, false, false, false>(a, m, x, y, z, n, fb, gb);
    else if (a.per[0])
      tgather<L, R, M, true, false, false, true>(a, m, x, y, z, n, fb, gb);
    else
      tgather<L, R, M, true, false, false>(a, m, x, y, z, n, fb, gb);
  } else {
    tgather<L, R, M, true, true, D == 3>(a, m, x, y, z, n, fb, gb);
  }
  add_seed<L, R, UP>(t, a.c, A.dJdT ? A.dJdT[node] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP, false, L::Qg>(t, a.c, fb, gb);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) s += (double)(wg[q] * gb[q]);
  A.dTinit[node] = s;
}

template <class L, class R, int UP>
hipError_t launch_adj(const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  constexpr int D = L::D;
  const StepArgs<R>& a = step ? step->s : init->s;
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  const dim3 block(bx, by, 1);
  const dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (step) {
    constexpr int Q = L::Qf + L::Qg;
    const double bytes = (double)a.nxp * a.ny * a.nz * Q * sizeof(R);
    // the standard-rate specialisation: for every pair in FP32, and for the
    // D2Q5 / D3Q7 pairs in FP64 (the paper's lattices in FP64 hold about 256
    // VGPRs either way, and the specialisation doubles their compile time)
    constexpr bool kStd = L::Qg == 2 * D + 1 || sizeof(R) == 4;
    const bool std_rates = kStd && standard_rates(a, D, L::Qg);
    if constexpr (D == 3 && sizeof(R) == 4) {
      if (bytes < 4294967296.0) {
        if constexpr (kStd) {
          if (std_rates) {
            adjoint_step_kernel_3f<L, Buf32<R, Q>, UP, true><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
            return hipGetLastError();
          }
        }
        adjoint_step_kernel_3f<L, Buf32<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
      } else {
        adjoint_step_kernel_3f<L, Glob64<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, 0u);
      }
    } else {
      if (bytes < 4294967296.0) {
        if constexpr (kStd) {
          if (std_rates) {
            adjoint_step_kernel<L, R, Buf32<R, Q>, UP, true><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
            return hipGetLastError();
          }
        }
        adjoint_step_kernel<L, R, Buf32<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, (unsigned)bytes);
      } else {
        adjoint_step_kernel<L, R, Glob64<R, Q>, UP, false><<<grid, block, 0, st>>>(*step, 0u);
      }
    }
  } else {
    adjoint_init_kernel<L, R, UP><<<grid, block, 0, st>>>(*init);
  }
  return hipGetLastError();
}

// Launchers of the D3Q27 + D3Q7 pair and of the paper's thermal lattices (one
// source file each).
template <class R>
hipError_t launch_adj_d3q7(int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st);
template <class R>
hipError_t launch_adj_d2q9(int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st);
template <class R>
hipError_t launch_adj_d3q15(int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st);

}  // namespace adjk
}  // namespace fpc
