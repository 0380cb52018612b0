// Batched (ensemble) 2-D stage kernels, element type double, the HLLC flux.
#include "batch_launch.h"

namespace snap {

int batched_occupancy_hllc_f64(int ntracer, int v) {
  return batch_occ_t<double, false, true>(ntracer, v);
}

int launch_stage2d_batched_hllc_f64(int ntracer, int v, const StageArgs* d, const int* first,
                                    int n, int nb, hipStream_t st) {
  return batch_launch_t<double, false, true>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
