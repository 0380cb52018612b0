// Batched (ensemble) 2-D stage kernels, element type double.
#include "batch_launch.h"

namespace snap {

TileShape batched_tile_f64(int ntracer, int v) { return batch_tile_t<double>(ntracer, v); }

int batched_occupancy_f64(int ntracer, int v) { return batch_occ_t<double>(ntracer, v); }

int launch_stage2d_batched_f64(int ntracer, int v, const StageArgs* d, const int* first, int n,
                              int nb, hipStream_t st) {
  return batch_launch_t<double>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
