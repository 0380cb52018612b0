// Adjoint kernels with the HLLC flux, single precision (conserved -> primitive reverse in double).
#include "adjoint_launch.h"

namespace snap {

int launch_adj_rhs_hllc_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                            void* out, int mode, double alpha, double beta, const void* y,
                            double gam, hipStream_t st) {
  return adj_rhs_t<float, true, false>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
}

}  // namespace snap
