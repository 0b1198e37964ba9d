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
#include "fpc_adjoint.h"
#include "fpc_kernels.h"

namespace fpc {
namespace {

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

// Source of link (ex, ey, ez) pulled at (x, y, z): returns false for a wall
// link (then `face` is the face crossed if exactly one), true otherwise with
// the wrapped source node in `src`.
template <class R>
__device__ __forceinline__ bool link_source(const StepArgs<R>& a, int x, int y, int z, int ex, int ey, int ez,
                                            unsigned& src, int& ncross, int& face) {
  int c[3] = {x - ex, y - ey, z - ez};
  const int n[3] = {a.nx, a.ny, a.nz};
  const int e[3] = {ex, ey, ez};
  ncross = 0;
  face = -1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (e[k] != 0 && (c[k] < 0 || c[k] >= n[k])) {
      if (a.per[k]) {
        c[k] = c[k] < 0 ? n[k] - 1 : 0;
      } else {
        ++ncross;
        face = 2 * k + (c[k] < 0 ? 0 : 1);
      }
    }
  }
  src = ((unsigned)c[2] * (unsigned)a.ny + (unsigned)c[1]) * (unsigned)a.nx + (unsigned)c[0];
  return ncross == 0;
}

__device__ __forceinline__ size_t profile_index(int face, int x, int y, int z, int nx, int ny) {
  const int k = face >> 1;
  return k == 0 ? (size_t)z * ny + y : (k == 1 ? (size_t)z * nx + x : (size_t)y * nx + x);
}

template <class R, int D>
__device__ __forceinline__ double face_temperature(const StepArgs<R>& a, int F, int x, int y, int z) {
  double Tw = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (f == F) Tw = a.face[f].Tprof ? a.face[f].Tprof[profile_index(f, x, y, z, a.nx, a.ny)] : a.face[f].Tw;
  return Tw;
}

template <class R>
__device__ __forceinline__ void face_flags(const StepArgs<R>& a, int F, bool& lid, bool& dir, double uw[3]) {
  lid = false;
  dir = false;
  uw[0] = uw[1] = uw[2] = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (f == F) {
      lid = a.face[f].lid;
      dir = a.face[f].dirichlet;
      uw[0] = a.face[f].uw[0];
      uw[1] = a.face[f].uw[1];
      uw[2] = a.face[f].uw[2];
    }
}

// Pulled populations of node (x, y, z) as plain values (storage offsets added).
template <class R, int D>
__device__ void pull_plain(const StepArgs<R>& a, int x, int y, int z, unsigned node, R* f, R* g) {
  using Lk = LinkOf<D>;
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) {
    unsigned src;
    int nc, F;
    R v;
    if (link_source(a, x, y, z, Lk::ex(q), Lk::ey(q), Lk::ez(q), src, nc, F)) {
      v = a.src[(size_t)q * a.plane + src];
    } else {
      v = a.src[(size_t)Lk::opp(q) * a.plane + node];
      bool lid, dir;
      double uw[3];
      face_flags(a, F, lid, dir, uw);
      if (nc == 1 && lid)
        v += R(2.0 * 3.0 * Lk::w(q)) * a.rho_w * R(Lk::ex(q) * uw[0] + Lk::ey(q) * uw[1] + Lk::ez(q) * uw[2]);
    }
    f[q] = v + R(Lk::w(q)) * a.c.rho_r;
  }
  const R Tr = tref(a, x, y, z);
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) {
    unsigned src;
    int nc, F;
    R v;
    const R wq = q == 0 ? R(1) - R(D) * a.c.cs2T : R(0.5) * a.c.cs2T;
    if (link_source(a, x, y, z, Lk::ex(q), Lk::ey(q), Lk::ez(q), src, nc, F)) {
      // stored against the source node's reference Tr(x - e)
      const R Trs = Tr - (R(Lk::ex(q)) * a.Tg[0] + R(Lk::ey(q)) * a.Tg[1] + R(Lk::ez(q)) * a.Tg[2]);
      v = a.src[(size_t)(Lk::Qf + q) * a.plane + src] + wq * Trs;
    } else {
      v = a.src[(size_t)(Lk::Qf + Lk::opp(q)) * a.plane + node] + wq * Tr;
      bool lid, dir;
      double uw[3];
      face_flags(a, F, lid, dir, uw);
      if (dir) v = -v + a.c.cs2T * R(face_temperature<R, D>(a, F, x, y, z));
    }
    g[q] = v;
  }
}

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

template <int D, class R, int UP>
__global__ void __launch_bounds__(256) adjoint_step_kernel(AdjArgs<R> A) {
  using Lk = LinkOf<D>;
  const StepArgs<R>& a = A.s;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const unsigned node = ((unsigned)z * (unsigned)a.ny + (unsigned)y) * (unsigned)a.nx + (unsigned)x;
  R f[Lk::Qf], g[Lk::Qg];
  pull_plain<R, D>(a, x, y, z, node, f, g);
  adj::Tape<R, D> t;
  adj::forward<R, D, UP>(f, g, a.c, t);
  R fb[Lk::Qf], gb[Lk::Qg];
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) fb[q] = A.lam_in[(size_t)q * a.plane + node];
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) gb[q] = A.lam_in[(size_t)(Lk::Qf + q) * a.plane + node];
  add_seed<R, D, UP>(t, a.c, A.dJdT ? A.dJdT[node] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP>(t, a.c, fb, gb);
  // push the link adjoints to the slots they were pulled from
#pragma unroll
  for (int q = 0; q < Lk::Qf; ++q) {
    unsigned src;
    int nc, F;
    if (link_source(a, x, y, z, Lk::ex(q), Lk::ey(q), Lk::ez(q), src, nc, F))
      A.lam_out[(size_t)q * a.plane + src] = fb[q];
    else
      A.lam_out[(size_t)Lk::opp(q) * a.plane + node] = fb[q];
  }
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) {
    unsigned src;
    int nc, F;
    if (link_source(a, x, y, z, Lk::ex(q), Lk::ey(q), Lk::ez(q), src, nc, F)) {
      A.lam_out[(size_t)(Lk::Qf + q) * a.plane + src] = gb[q];
    } else {
      bool lid, dir;
      double uw[3];
      face_flags(a, F, lid, dir, uw);
      A.lam_out[(size_t)(Lk::Qf + Lk::opp(q)) * a.plane + node] = dir ? -gb[q] : gb[q];
      if (dir) {
        double* dt = nullptr;
#pragma unroll
        for (int ff = 0; ff < 6; ++ff)
          if (ff == F) dt = A.dtheta[ff];
        if (dt) dt[profile_index(F, x, y, z, a.nx, a.ny)] += (double)(a.c.cs2T * gb[q]);
      }
    }
  }
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
  const unsigned node = ((unsigned)z * (unsigned)a.ny + (unsigned)y) * (unsigned)a.nx + (unsigned)x;
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
  for (int q = 0; q < Lk::Qf; ++q) fb[q] = A.lam0[(size_t)q * a.plane + node];
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) gb[q] = A.lam0[(size_t)(Lk::Qf + q) * a.plane + node];
  add_seed<R, D, UP>(t, a.c, A.dJdT ? A.dJdT[node] : 0.0, A.ke, fb, gb);
  adj::reverse<R, D, UP>(t, a.c, fb, gb);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < Lk::Qg; ++q) s += (double)(wg[q] * gb[q]);
  A.dTinit[node] = s;
}

template <int D, class R, int UP>
hipError_t launch_adj(const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  const StepArgs<R>& a = step ? step->s : init->s;
  const int bx = a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64);
  const int by = 256 / bx;
  const dim3 block(bx, by, 1);
  const dim3 grid((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
  if (step)
    adjoint_step_kernel<D, R, UP><<<grid, block, 0, st>>>(*step);
  else
    adjoint_init_kernel<D, R, UP><<<grid, block, 0, st>>>(*init);
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
