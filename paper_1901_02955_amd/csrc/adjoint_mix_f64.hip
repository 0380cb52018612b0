// Adjoint kernels under the mixture equation of state, double precision.
#include "adjoint_launch.h"

namespace snap {

int launch_adj_rhs_mix_f64(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                           void* out, int mode, double alpha, double beta, const void* y,
                           double gam, hipStream_t st) {
  return adj_rhs_t<double, false, true>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
}

}  // namespace snap
