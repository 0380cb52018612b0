// Stage kernels, single precision storage and stencil arithmetic, mixture
// equation of state (tracers >= 1; the conserved -> primitive conversion stays
// in double).
#include "stage_launch.h"

namespace snap {

int launch_stage_mix_f32(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st) {
  return launch_stage_t<float, true>(ntracer, d3, a, nblocks, st);
}

int occupancy_mix_f32(int ntracer, bool d3) { return occupancy_t<float, true>(ntracer, d3); }

}  // namespace snap
