// Stage kernels without tracers, element type double: the dry-gas forms of the
// LMARS and HLLC kernels. build.py compiles this file with the iterative ILP
// scheduling strategy, which makes these kernels faster at the same occupancy;
// the kernels with tracers keep the default strategy, under which several of
// them hold one more wave per SIMD.
#include "stage_launch.h"

namespace snap {

int launch_stage_dry_f64(bool hllc, bool d3, const StageArgs& a, int nblocks, hipStream_t st) {
  return hllc ? launch_nt<double, 0, false, true>(d3, a, nblocks, st)
              : launch_nt<double, 0, false, false>(d3, a, nblocks, st);
}

int occupancy_dry_f64(bool hllc, bool d3) {
  return hllc ? occupancy_nt<double, 0, false, true>(d3) : occupancy_nt<double, 0, false, false>(d3);
}

}  // namespace snap
