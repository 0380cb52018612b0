// Batched (ensemble) 2-D stage kernels, element type double.
#include "batch_launch.h"

namespace snap {

int batched_occupancy_mix_f64(int ntracer, int v);
int batched_occupancy_hllc_f64(int ntracer, int v);
int launch_stage2d_batched_mix_f64(int ntracer, int v, const StageArgs* d, const int* first, int n,
                                  int nb, hipStream_t st);
int launch_stage2d_batched_hllc_f64(int ntracer, int v, const StageArgs* d, const int* first,
                                   int n, int nb, hipStream_t st);

TileShape batched_tile_f64(int ntracer, int v) { return batch_tile_t<double>(ntracer, v); }

// form: 0 passive tracers with LMARS; 1 the mixture (batch_mix_f64.hip);
// 2 HLLC (batch_hllc_f64.hip)
int batched_occupancy_f64(int ntracer, int v, int form) {
  if (form == 1) return batched_occupancy_mix_f64(ntracer, v);
  if (form == 2) return batched_occupancy_hllc_f64(ntracer, v);
  return batch_occ_t<double, false, false>(ntracer, v);
}

int launch_stage2d_batched_f64(int ntracer, int v, int form, const StageArgs* d, const int* first,
                              int n, int nb, hipStream_t st) {
  if (form == 1) return launch_stage2d_batched_mix_f64(ntracer, v, d, first, n, nb, st);
  if (form == 2) return launch_stage2d_batched_hllc_f64(ntracer, v, d, first, n, nb, st);
  return batch_launch_t<double, false, false>(ntracer, v, d, first, n, nb, st);
}

}  // namespace snap
