// Instantiation and dispatch of the stage kernels for one element type.
// Included by the stage_*.hip files, one per element type and kernel family,
// so that the instantiation sets compile in parallel.
#pragma once

#include "snap_internal.h"

namespace snap {

// Tile shape per element type and variable count: the largest of 16 x 16,
// 16 x 8 and 8 x 8 whose LDS plane stays within 56 KiB, so that at least two
// (usually three) workgroups share a compute unit's 160 KiB of LDS.
template <typename T, int NT>
struct TileFor {
  static constexpr int NV = 5 + NT;
  static constexpr bool BIG = sizeof(Plane<T, NV, 16, 16>) <= 56 * 1024;
  static constexpr bool MID = sizeof(Plane<T, NV, 16, 8>) <= 56 * 1024;
#if defined(SNAP_TILE_X) && defined(SNAP_TILE_Y)
  static constexpr int TX = NT == 0 ? SNAP_TILE_X : (BIG || MID ? 16 : 8);
  static constexpr int TY = NT == 0 ? SNAP_TILE_Y : (BIG ? 16 : 8);
#else
  static constexpr int TX = BIG || MID ? 16 : 8;
  static constexpr int TY = BIG ? 16 : 8;
#endif
};

// MIX: the mixture equation of state (instantiated for NT >= 1 only; with no
// tracers the mixture is the dry gas). HLLC: the HLLC Riemann solver (passive
// tracers).
template <typename T, int NT, bool MIX, bool HLLC = false>
int launch_nt(bool d3, const StageArgs& a, int nblocks, hipStream_t st) {
  constexpr int TX = TileFor<T, NT>::TX, TY = TileFor<T, NT>::TY;
  constexpr bool M = MIX && NT > 0;
  if (d3)
    hipLaunchKernelGGL((k_stage3d<T, NT, TX, TY, M, HLLC>), dim3(nblocks), dim3(TX * TY), 0, st,
                       a);
  else
    hipLaunchKernelGGL((k_stage2d<T, NT, TX, TY, M, HLLC>), dim3(nblocks), dim3(TX * TY), 0, st,
                       a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int NT, bool MIX, bool HLLC = false>
int occupancy_nt(bool d3) {
  constexpr int TX = TileFor<T, NT>::TX, TY = TileFor<T, NT>::TY;
  constexpr bool M = MIX && NT > 0;
  int n = 0;
  const void* k = d3 ? reinterpret_cast<const void*>(&k_stage3d<T, NT, TX, TY, M, HLLC>)
                     : reinterpret_cast<const void*>(&k_stage2d<T, NT, TX, TY, M, HLLC>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, TX * TY, 0) != hipSuccess) return 0;
  return n;
}

// 3-D stage kernels with the sedimentation terms (mixture, NT >= 1).
template <typename T, int NT>
int launch_sed_nt(const StageArgs& a, int nblocks, hipStream_t st) {
  constexpr int TX = TileFor<T, NT>::TX, TY = TileFor<T, NT>::TY;
  hipLaunchKernelGGL((k_stage3d<T, NT, TX, TY, true, false, true>), dim3(nblocks), dim3(TX * TY),
                     0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int NT>
int occupancy_sed_nt() {
  constexpr int TX = TileFor<T, NT>::TX, TY = TileFor<T, NT>::TY;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(&k_stage3d<T, NT, TX, TY, true, false, true>),
          TX * TY, 0) != hipSuccess)
    return 0;
  return n;
}

template <typename T>
int launch_sed_t(int ntracer, const StageArgs& a, int nblocks, hipStream_t st) {
  switch (ntracer) {
    case 1: return launch_sed_nt<T, 1>(a, nblocks, st);
    case 2: return launch_sed_nt<T, 2>(a, nblocks, st);
    case 3: return launch_sed_nt<T, 3>(a, nblocks, st);
    case 4: return launch_sed_nt<T, 4>(a, nblocks, st);
    case 5: return launch_sed_nt<T, 5>(a, nblocks, st);
    case 6: return launch_sed_nt<T, 6>(a, nblocks, st);
    case 7: return launch_sed_nt<T, 7>(a, nblocks, st);
    case 8: return launch_sed_nt<T, 8>(a, nblocks, st);
    default: return -1;
  }
}

template <typename T>
int occupancy_sed_t(int ntracer) {
  switch (ntracer) {
    case 1: return occupancy_sed_nt<T, 1>();
    case 2: return occupancy_sed_nt<T, 2>();
    case 3: return occupancy_sed_nt<T, 3>();
    case 4: return occupancy_sed_nt<T, 4>();
    case 5: return occupancy_sed_nt<T, 5>();
    case 6: return occupancy_sed_nt<T, 6>();
    case 7: return occupancy_sed_nt<T, 7>();
    case 8: return occupancy_sed_nt<T, 8>();
    default: return 0;
  }
}

// Without tracers the mixture is the dry gas, and the kernels are the ones of
// stage_dry_f64.hip / stage_dry_f32.hip, so that no other translation unit
// instantiates them.
template <typename T>
int launch_dry(bool hllc, bool d3, const StageArgs& a, int nblocks, hipStream_t st) {
  if constexpr (sizeof(T) == 8)
    return launch_stage_dry_f64(hllc, d3, a, nblocks, st);
  else
    return launch_stage_dry_f32(hllc, d3, a, nblocks, st);
}

template <typename T>
int occupancy_dry(bool hllc, bool d3) {
  if constexpr (sizeof(T) == 8)
    return occupancy_dry_f64(hllc, d3);
  else
    return occupancy_dry_f32(hllc, d3);
}

// Workgroups of the stage kernel that fit on one compute unit (0 if unknown).
template <typename T, bool MIX, bool HLLC = false>
int occupancy_t(int ntracer, bool d3) {
  switch (ntracer) {
    case 0: return occupancy_dry<T>(HLLC, d3);
    case 1: return occupancy_nt<T, 1, MIX, HLLC>(d3);
    case 2: return occupancy_nt<T, 2, MIX, HLLC>(d3);
    case 3: return occupancy_nt<T, 3, MIX, HLLC>(d3);
    case 4: return occupancy_nt<T, 4, MIX, HLLC>(d3);
    case 5: return occupancy_nt<T, 5, MIX, HLLC>(d3);
    case 6: return occupancy_nt<T, 6, MIX, HLLC>(d3);
    case 7: return occupancy_nt<T, 7, MIX, HLLC>(d3);
    case 8: return occupancy_nt<T, 8, MIX, HLLC>(d3);
    default: return 0;
  }
}

template <typename T, bool MIX, bool HLLC = false>
int launch_stage_t(int ntracer, bool d3, const StageArgs& a, int nblocks, hipStream_t st) {
  switch (ntracer) {
    case 0: return launch_dry<T>(HLLC, d3, a, nblocks, st);
    case 1: return launch_nt<T, 1, MIX, HLLC>(d3, a, nblocks, st);
    case 2: return launch_nt<T, 2, MIX, HLLC>(d3, a, nblocks, st);
    case 3: return launch_nt<T, 3, MIX, HLLC>(d3, a, nblocks, st);
    case 4: return launch_nt<T, 4, MIX, HLLC>(d3, a, nblocks, st);
    case 5: return launch_nt<T, 5, MIX, HLLC>(d3, a, nblocks, st);
    case 6: return launch_nt<T, 6, MIX, HLLC>(d3, a, nblocks, st);
    case 7: return launch_nt<T, 7, MIX, HLLC>(d3, a, nblocks, st);
    case 8: return launch_nt<T, 8, MIX, HLLC>(d3, a, nblocks, st);
    default: return -1;
  }
}

template <typename T>
TileShape tile_t(int nv) {
  switch (nv - 5) {
    case 0: return {TileFor<T, 0>::TX, TileFor<T, 0>::TY};
    case 1: return {TileFor<T, 1>::TX, TileFor<T, 1>::TY};
    case 2: return {TileFor<T, 2>::TX, TileFor<T, 2>::TY};
    case 3: return {TileFor<T, 3>::TX, TileFor<T, 3>::TY};
    case 4: return {TileFor<T, 4>::TX, TileFor<T, 4>::TY};
    case 5: return {TileFor<T, 5>::TX, TileFor<T, 5>::TY};
    case 6: return {TileFor<T, 6>::TX, TileFor<T, 6>::TY};
    case 7: return {TileFor<T, 7>::TX, TileFor<T, 7>::TY};
    default: return {TileFor<T, 8>::TX, TileFor<T, 8>::TY};
  }
}

}  // namespace snap
