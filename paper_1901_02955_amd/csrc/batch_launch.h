// Tile variants and dispatch of the batched (ensemble) 2-D stage kernel for one
// element type and form (MIX: the mixture equation of state; HLLC: the HLLC
// flux; neither: passive tracers with LMARS). Variant 0 is the single-domain
// default shape; variants 1..5 (ntracer == 0 only) are alternatives for the
// autotuner. A variant whose LDS plane would exceed 64 KiB is unavailable.
#pragma once

#include "stage_launch.h"

namespace snap {

template <int V>
struct BatchShape;
template <> struct BatchShape<1> { static constexpr int TX = 32, TZ = 8; };
template <> struct BatchShape<2> { static constexpr int TX = 64, TZ = 4; };
template <> struct BatchShape<3> { static constexpr int TX = 8, TZ = 32; };
template <> struct BatchShape<4> { static constexpr int TX = 16, TZ = 8; };
template <> struct BatchShape<5> { static constexpr int TX = 32, TZ = 16; };

template <typename T, int NT, int TX, int TZ>
constexpr bool batch_fits() {
  return sizeof(Plane<T, 5 + NT, TX, TZ>) <= 64 * 1024;
}

template <typename T, int NT, int TX, int TZ, bool MIX, bool HLLC>
int batch_launch_shape(const StageArgs* d, const int* first, int n, int nblocks, hipStream_t st) {
  if constexpr (!batch_fits<T, NT, TX, TZ>() || (MIX && NT == 0)) {
    return -2;
  } else {
    hipLaunchKernelGGL((k_stage2d_batched<T, NT, TX, TZ, MIX, HLLC>), dim3(nblocks), dim3(TX * TZ),
                       0, st, d, first, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
}

template <typename T, int NT, int TX, int TZ, bool MIX, bool HLLC>
int batch_occ_shape() {
  if constexpr (!batch_fits<T, NT, TX, TZ>() || (MIX && NT == 0)) {
    return 0;
  } else {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&k_stage2d_batched<T, NT, TX, TZ, MIX, HLLC>),
            TX * TZ, 0) != hipSuccess)
      return 0;
    return nb;
  }
}

template <typename T, int NT>
TileShape batch_tile_nt(int v) {
  if constexpr (NT != 0) return TileShape{TileFor<T, NT>::TX, TileFor<T, NT>::TY};
  switch (v) {
#define SNAP_BSHAPE(V)                                                              \
  case V:                                                                           \
    return batch_fits<T, NT, BatchShape<V>::TX, BatchShape<V>::TZ>()                \
               ? TileShape{BatchShape<V>::TX, BatchShape<V>::TZ}                    \
               : TileShape{0, 0};
    SNAP_BSHAPE(1)
    SNAP_BSHAPE(2)
    SNAP_BSHAPE(3)
    SNAP_BSHAPE(4)
    SNAP_BSHAPE(5)
#undef SNAP_BSHAPE
    default: return TileShape{TileFor<T, NT>::TX, TileFor<T, NT>::TY};
  }
}

template <typename T, int NT, bool MIX, bool HLLC>
int batch_launch_nt(int v, const StageArgs* d, const int* first, int n, int nb, hipStream_t st) {
  if constexpr (NT == 0) {
    switch (v) {
      case 1: return batch_launch_shape<T, NT, 32, 8, MIX, HLLC>(d, first, n, nb, st);
      case 2: return batch_launch_shape<T, NT, 64, 4, MIX, HLLC>(d, first, n, nb, st);
      case 3: return batch_launch_shape<T, NT, 8, 32, MIX, HLLC>(d, first, n, nb, st);
      case 4: return batch_launch_shape<T, NT, 16, 8, MIX, HLLC>(d, first, n, nb, st);
      case 5: return batch_launch_shape<T, NT, 32, 16, MIX, HLLC>(d, first, n, nb, st);
      default: break;
    }
  }
  return batch_launch_shape<T, NT, TileFor<T, NT>::TX, TileFor<T, NT>::TY, MIX, HLLC>(d, first, n,
                                                                                     nb, st);
}

template <typename T, int NT, bool MIX, bool HLLC>
int batch_occ_nt(int v) {
  if constexpr (NT == 0) {
    switch (v) {
      case 1: return batch_occ_shape<T, NT, 32, 8, MIX, HLLC>();
      case 2: return batch_occ_shape<T, NT, 64, 4, MIX, HLLC>();
      case 3: return batch_occ_shape<T, NT, 8, 32, MIX, HLLC>();
      case 4: return batch_occ_shape<T, NT, 16, 8, MIX, HLLC>();
      case 5: return batch_occ_shape<T, NT, 32, 16, MIX, HLLC>();
      default: break;
    }
  }
  return batch_occ_shape<T, NT, TileFor<T, NT>::TX, TileFor<T, NT>::TY, MIX, HLLC>();
}

#define SNAP_NT_SWITCH(CALL)        \
  switch (ntracer) {                \
    case 0: return CALL(0);         \
    case 1: return CALL(1);         \
    case 2: return CALL(2);         \
    case 3: return CALL(3);         \
    case 4: return CALL(4);         \
    case 5: return CALL(5);         \
    case 6: return CALL(6);         \
    case 7: return CALL(7);         \
    case 8: return CALL(8);         \
    default: break;                 \
  }

template <typename T>
TileShape batch_tile_t(int ntracer, int v) {
  if (ntracer != 0 && v != 0) return TileShape{0, 0};
#define SNAP_CALL(NT) batch_tile_nt<T, NT>(v)
  SNAP_NT_SWITCH(SNAP_CALL)
#undef SNAP_CALL
  return TileShape{0, 0};
}

template <typename T, bool MIX, bool HLLC>
int batch_launch_t(int ntracer, int v, const StageArgs* d, const int* first, int n, int nb,
                   hipStream_t st) {
#define SNAP_CALL(NT) batch_launch_nt<T, NT, MIX, HLLC>(v, d, first, n, nb, st)
  SNAP_NT_SWITCH(SNAP_CALL)
#undef SNAP_CALL
  return -1;
}

template <typename T, bool MIX, bool HLLC>
int batch_occ_t(int ntracer, int v) {
#define SNAP_CALL(NT) batch_occ_nt<T, NT, MIX, HLLC>(v)
  SNAP_NT_SWITCH(SNAP_CALL)
#undef SNAP_CALL
  return 0;
}

}  // namespace snap
