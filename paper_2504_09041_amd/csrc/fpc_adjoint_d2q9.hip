// Adjoint kernels of the paper's D2Q9 thermal lattice (Sec. 4.4, App. B); the
// kernels are those of fpc_adjoint_kernels.h, instantiated here so that the
// lattice groups compile in parallel.
#include "fpc_adjoint_kernels.h"

namespace fpc {
namespace adjk {

template <class R>
hipError_t launch_adj_d2q9(int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  return up == 0 ? launch_adj<Lat2T9, R, 0>(step, init, st) : launch_adj<Lat2T9, R, 1>(step, init, st);
}

template hipError_t launch_adj_d2q9<double>(int, const AdjArgs<double>*, const AdjInitArgs<double>*, hipStream_t);
template hipError_t launch_adj_d2q9<float>(int, const AdjArgs<float>*, const AdjInitArgs<float>*, hipStream_t);

}  // namespace adjk
}  // namespace fpc
