// Adjoint kernels, single precision (conserved -> primitive reverse in double).
#include "adjoint_launch.h"

namespace snap {

// the HLLC instances (adjoint_hllc_f32.hip)
int launch_adj_rhs_hllc_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                            void* out, int mode, double alpha, double beta, const void* y,
                            double gam, hipStream_t st);

int launch_adj_rhs_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                       void* out, int mode, double alpha, double beta, const void* y, double gam,
                       hipStream_t st) {
  if (a.hllc) return launch_adj_rhs_hllc_f32(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
  return adj_rhs_t<float, false>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
}

}  // namespace snap
