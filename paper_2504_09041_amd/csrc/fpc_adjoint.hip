// Adjoint stream-collide step and adjoint of the initial collision: the
// launchers of the C ABI, and the kernels of the D2Q9 + D2Q5 pair (the
// kernels themselves: fpc_adjoint_kernels.h; the other pairs are instantiated
// in fpc_adjoint_d3q7.hip, fpc_adjoint_d2q9.hip and fpc_adjoint_d3q15.hip).
#include "fpc_adjoint_kernels.h"

namespace fpc {
namespace adjk {
namespace {

// tk: thermal lattice, 0 = D2Q5 / D3Q7, 1 = the paper's D2Q9 / D3Q15
template <class R>
hipError_t dispatch(int dim, int up, int tk, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  if (tk == 1) return dim == 2 ? launch_adj_d2q9<R>(up, step, init, st) : launch_adj_d3q15<R>(up, step, init, st);
  if (dim == 3) return launch_adj_d3q7<R>(up, step, init, st);
  return up == 0 ? launch_adj<Lat2, R, 0>(step, init, st) : launch_adj<Lat2, R, 1>(step, init, st);
}

}  // namespace
}  // namespace adjk

using adjk::AdjArgs;
using adjk::AdjInitArgs;
using adjk::dispatch;

template <class R>
hipError_t launch_adjoint_step(const StepArgs<R>& a, int dim, int up, int tk, const void* lam_in, void* lam_out,
                               const double* dJdT, double ke, double* const dtheta[6], hipStream_t st) {
  AdjArgs<R> A;
  A.s = a;
  A.lam_in = static_cast<const R*>(lam_in);
  A.lam_out = static_cast<R*>(lam_out);
  A.dJdT = dJdT;
  A.ke = ke;
  for (int f = 0; f < 6; ++f) A.dtheta[f] = dtheta ? dtheta[f] : nullptr;
  return dispatch<R>(dim, up, tk, &A, nullptr, st);
}

template <class R>
hipError_t launch_adjoint_init(const StepArgs<R>& a, int dim, int up, int tk, const double* T_init, const void* lam0,
                               const double* dJdT, double ke, double* dTinit, hipStream_t st) {
  AdjInitArgs<R> A;
  A.s = a;
  A.T_init = T_init;
  A.lam0 = static_cast<const R*>(lam0);
  A.dJdT = dJdT;
  A.ke = ke;
  A.dTinit = dTinit;
  return dispatch<R>(dim, up, tk, nullptr, &A, st);
}

template hipError_t launch_adjoint_step<double>(const StepArgs<double>&, int, int, int, const void*, void*,
                                                const double*, double, double* const[6], hipStream_t);
template hipError_t launch_adjoint_step<float>(const StepArgs<float>&, int, int, int, const void*, void*,
                                               const double*, double, double* const[6], hipStream_t);
template hipError_t launch_adjoint_init<double>(const StepArgs<double>&, int, int, int, const double*, const void*,
                                                const double*, double, double*, hipStream_t);
template hipError_t launch_adjoint_init<float>(const StepArgs<float>&, int, int, int, const double*, const void*,
                                               const double*, double, double*, hipStream_t);

}  // namespace fpc
