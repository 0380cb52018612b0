// Adjoint kernels, single precision (conserved -> primitive reverse in double).
#include "adjoint_launch.h"

namespace snap {

int launch_adj_rhs_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                       void* out, int mode, double alpha, double beta, hipStream_t st) {
  return adj_rhs_t<float>(w, a, q, rb, out, mode, alpha, beta, st);
}

int launch_adj_combine_f32(void* out, const void* x, const void* y, const void* z, double ca,
                           double cb, double cc, long long n, hipStream_t st) {
  return adj_combine_t<float>(out, x, y, z, ca, cb, cc, n, st);
}

}  // namespace snap
