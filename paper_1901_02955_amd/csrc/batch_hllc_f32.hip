// Batched (ensemble) 2-D stage kernels, element type float, the HLLC flux.
#include "batch_launch.h"

namespace snap {

int batched_occupancy_hllc_f32(int ntracer, int v) {
  return batch_occ_t<float, false, true>(ntracer, v);
}

int launch_stage2d_batched_hllc_f32(int ntracer, int v, const StageArgs* d, const int* first,
                                    int n, int nb, hipStream_t st) {
  return batch_launch_t<float, false, true>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
