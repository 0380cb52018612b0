// Batched (ensemble) 2-D stage kernels, element type double, the mixture equation of state.
#include "batch_launch.h"

namespace snap {

int batched_occupancy_mix_f64(int ntracer, int v) {
  return batch_occ_t<double, true, false>(ntracer, v);
}

int launch_stage2d_batched_mix_f64(int ntracer, int v, const StageArgs* d, const int* first,
                                   int n, int nb, hipStream_t st) {
  return batch_launch_t<double, true, false>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
