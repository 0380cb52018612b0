// Stage kernels, double precision, mixture equation of state (tracers >= 1).
#include "stage_launch.h"

namespace snap {

int launch_stage_mix_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st) {
  return launch_stage_t<double, true>(ntracer, d3, a, nblocks, st);
}

int occupancy_mix_f64(int ntracer, bool d3) { return occupancy_t<double, true>(ntracer, d3); }

}  // namespace snap
