// Batched (ensemble) 2-D stage kernels, element type float.
#include "batch_launch.h"

namespace snap {

TileShape batched_tile_f32(int ntracer, int v) { return batch_tile_t<float>(ntracer, v); }

int batched_occupancy_f32(int ntracer, int v) { return batch_occ_t<float>(ntracer, v); }

int launch_stage2d_batched_f32(int ntracer, int v, const StageArgs* d, const int* first, int n,
                              int nb, hipStream_t st) {
  return batch_launch_t<float>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
