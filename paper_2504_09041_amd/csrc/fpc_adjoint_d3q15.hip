// Adjoint kernels of the paper's D3Q15 thermal lattice (Sec. 5.4, App. C); the
// kernels are those of fpc_adjoint_kernels.h, instantiated here so that the
// lattice groups compile in parallel.
#include "fpc_adjoint_kernels.h"

namespace fpc {
namespace adjk {

template <class R>
hipError_t launch_adj_d3q15(int up, const AdjArgs<R>* step, const AdjInitArgs<R>* init, hipStream_t st) {
  if (up == 0) return launch_adj<Lat3T15, R, 0>(step, init, st);
  if (up == 1) return launch_adj<Lat3T15, R, 1>(step, init, st);
  return launch_adj<Lat3T15, R, 2>(step, init, st);
}

// The build compiles this file once per storage precision, naming it in
// FPC_ADJ_REAL, so that the two compile in parallel; without the macro both
// are instantiated.
#ifdef FPC_ADJ_REAL
template hipError_t launch_adj_d3q15<FPC_ADJ_REAL>(int, const AdjArgs<FPC_ADJ_REAL>*, const AdjInitArgs<FPC_ADJ_REAL>*,
                                                   hipStream_t);
#else
template hipError_t launch_adj_d3q15<double>(int, const AdjArgs<double>*, const AdjInitArgs<double>*, hipStream_t);
template hipError_t launch_adj_d3q15<float>(int, const AdjArgs<float>*, const AdjInitArgs<float>*, hipStream_t);
#endif

}  // namespace adjk
}  // namespace fpc
