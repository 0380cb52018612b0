// Stage kernels, double precision, passive tracers.
#include "stage_launch.h"

namespace snap {

int launch_stage_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st) {
  return launch_stage_t<double, false>(ntracer, d3, a, nblocks, st);
}

TileShape tile_f64(int nv) { return tile_t<double>(nv); }

int occupancy_f64(int ntracer, bool d3) { return occupancy_t<double, false>(ntracer, d3); }

}  // namespace snap
