// Stage kernels with the HLLC Riemann solver, passive tracers, element type double.
#include "stage_launch.h"

namespace snap {

int launch_stage_hllc_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st) {
  return launch_stage_t<double, false, true>(ntracer, d3, a, nblocks, st);
}

int occupancy_hllc_f64(int ntracer, bool d3) { return occupancy_t<double, false, true>(ntracer, d3); }

}  // namespace snap
