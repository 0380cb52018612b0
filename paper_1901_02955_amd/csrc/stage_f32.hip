// Stage kernels, single precision storage and stencil arithmetic (the
// conserved -> primitive conversion and the reference state stay in double).
#include "stage_launch.h"

namespace snap {

int launch_stage_f32(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st) {
  return launch_stage_t<float, false>(ntracer, d3, a, nblocks, st);
}

TileShape tile_f32(int nv) { return tile_t<float>(nv); }

int occupancy_f32(int ntracer, bool d3) { return occupancy_t<float, false>(ntracer, d3); }

}  // namespace snap
