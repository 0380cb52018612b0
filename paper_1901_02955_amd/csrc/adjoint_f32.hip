// Adjoint kernels, single precision (conserved -> primitive reverse in double).
#include "adjoint_launch.h"

namespace snap {

// the HLLC and mixture instances (adjoint_hllc_f32.hip, adjoint_mix_f32.hip)
int launch_adj_rhs_hllc_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                            void* out, int mode, double alpha, double beta, const void* y,
                            double gam, hipStream_t st);
int launch_adj_rhs_mix_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                           void* out, int mode, double alpha, double beta, const void* y,
                           double gam, hipStream_t st);

int launch_adj_rhs_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                       void* out, int mode, double alpha, double beta, const void* y, double gam,
                       hipStream_t st) {
  if (a.hllc) return launch_adj_rhs_hllc_f32(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
  if (a.mixture) return launch_adj_rhs_mix_f32(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
  return adj_rhs_t<float, false, false>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
}

}  // namespace snap
