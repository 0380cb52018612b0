// 3-D stage kernels with falling condensates, single precision: the mixture
// kernels with the sedimentation terms added in their last phase.
#include "stage_launch.h"

namespace snap {

int launch_stage_sed_f32(int ntracer, const StageArgs& a, int nblocks, hipStream_t st) {
  return launch_sed_t<float>(ntracer, a, nblocks, st);
}

int occupancy_sed_f32(int ntracer) { return occupancy_sed_t<float>(ntracer); }

}  // namespace snap
