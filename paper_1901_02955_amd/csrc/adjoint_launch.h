// Dispatch of the adjoint kernels for one element type (included once per type).
#pragma once

#include <cstdlib>

#include "snap_adjoint.h"
#include "snap_internal.h"

namespace snap {

template <typename T, int NV, bool XDIR, bool HLLC, bool MIX>
void adj_line_launch(const T* q, const T* r, const AdjArgs& a, int d, T* P, hipStream_t st) {
  constexpr int LN = LineShape<T, NV, XDIR>::LN, TL = LineShape<T, NV, XDIR>::TL;
  const LineGeom g = line_geom(a, d);
  const long long blocks = ((g.nlines + LN - 1) / LN) * ((g.nd + TL - 1) / TL);
  hipLaunchKernelGGL((k_adj_line<T, NV, LN, TL, XDIR, HLLC, MIX>), dim3((unsigned)blocks),
                     dim3(LineTile<T, NV, LN, TL>::NTHR), 0,
                     st, q, r, a, d, P);
}

// The y and z directions march along their lines (k_adj_march) in single
// precision with up to 7 variables, where the march's register window fits,
// and where each variable's padded plane is smaller than 2 GiB; double
// precision, more variables and larger planes take the tiled kernel. Setting
// SNAP_ADJ_MARCH=0 selects the tiled kernel everywhere.
template <typename T, int NV>
constexpr bool march_fits() {
  return sizeof(T) == 4 && NV <= 7;
}

// (read at every launch, so that a process can compare both kernels)
inline bool march_enabled() {
  const char* e = getenv("SNAP_ADJ_MARCH");
  return !(e && e[0] == '0');
}

// The z march folds the cells at least 3 from the y and z edges, after
// k_adj_xmerge has added the x copies' cotangents into the cells within 3 of
// an x edge (the separate fold pass then covers the rows of the 3 lowest and 3
// highest levels and those within 3 of a y edge); SNAP_ADJ_MARCH_FOLD=0
// leaves every cell to the fold pass.
inline bool march_fold_enabled() {
  const char* e = getenv("SNAP_ADJ_MARCH_FOLD");
  return !(e && e[0] == '0');
}

// Segment length of the march: at most 43 cells, so that the 256 x 256 x 128
// grid gives 3 x 65536 z segments and 6 x 32768 y segments (three waves per
// SIMD of the 256 compute units, the kernel's occupancy with 5 variables),
// each recomputing a 3-cell halo on either side. On that grid one FP32
// right-hand-side adjoint took 1.100, 1.107, 1.085 and 1.133 ms with segments
// of 24, 32, 43 and 64 cells. SNAP_ADJ_MARCH_SEG overrides the length.
inline int march_seglen(int nd) {
  const char* e = getenv("SNAP_ADJ_MARCH_SEG");
  const int v = e ? atoi(e) : 0;
  const int target = v > 0 ? v : 43;
  const int nseg = (nd + target - 1) / target;
  return (nd + nseg - 1) / nseg;
}

template <typename T, int NV, int D, bool HLLC>
void adj_march_launch(const T* q, const T* r, const AdjArgs& a, T* P, const MarchFold<T>& fo,
                      hipStream_t st) {
  const int nd = D == 2 ? a.nz : a.ny;
  const long long lines = (long long)a.nx * (D == 2 ? a.ny : a.nz);
  const int seg = march_seglen(nd);
  const dim3 grid((unsigned)((lines + 255) / 256), (unsigned)((nd + seg - 1) / seg));
  hipLaunchKernelGGL((k_adj_march<T, NV, D, HLLC>), grid, dim3(256), 0, st, q, r, a, seg, P, fo);
}

template <typename T, int NV, bool HLLC, bool MIX>
int adj_rhs_nv(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb, void* out,
               int mode, double alpha, double beta, const void* y, double gam, hipStream_t st) {
  const T* qs = static_cast<const T*>(q);
  const T* r = static_cast<const T*>(rb);
  T* P = static_cast<T*>(w.P);
  adj_line_launch<T, NV, true, HLLC, MIX>(qs, r, a, 0, P, st);
  // the march addresses each variable's plane with 32-bit byte offsets
  const bool planes_small = a.sv * (long long)sizeof(T) < (1LL << 31) &&
                            a.rv * (long long)sizeof(T) < (1LL << 31);
  // (the mixture takes the tiled kernel in every direction)
  bool zfold = false;   // the z march folds the cells at least 3 from the y and z edges
  if (march_fits<T, NV>() && !MIX && march_enabled() && planes_small) {
    if constexpr (march_fits<T, NV>() && !MIX) {
      zfold = march_fold_enabled() && a.nz > 6;
      MarchFold<T> none{nullptr, nullptr, 0, T(0), T(0), T(0)};
      MarchFold<T> fo{static_cast<T*>(out), static_cast<const T*>(y), mode,
                      static_cast<T>(alpha), static_cast<T>(beta), static_cast<T>(gam)};
      if (zfold) {
        const long long n = (long long)(a.nx > 6 ? 6 : a.nx) * a.ny * a.nz;
        hipLaunchKernelGGL((k_adj_xmerge<T, NV>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, P, a);
      }
      if (a.d3) adj_march_launch<T, NV, 1, HLLC>(qs, r, a, P, none, st);
      adj_march_launch<T, NV, 2, HLLC>(qs, r, a, P, zfold ? fo : none, st);
    }
  } else {
    if (a.d3) adj_line_launch<T, NV, false, HLLC, MIX>(qs, r, a, 1, P, st);
    adj_line_launch<T, NV, false, HLLC, MIX>(qs, r, a, 2, P, st);
  }
  // falling condensates (mixture): the reverse of the sedimentation terms
  if constexpr (MIX) {
    if (a.sed.on) {
      const dim3 sgrid(a.ny * (a.nz + 2), (a.nx + 255) / 256);
      hipLaunchKernelGGL((k_adj_sediment<T, NV>), sgrid, dim3(256), 0, st, qs, r, a, P);
    }
  }
  // every row, or after a folding z march the rows it left
  const int ye = !a.d3 ? 0 : (a.ny > 6 ? 6 : a.ny);
  const int rows = zfold ? 6 * a.ny + (a.nz - 6) * ye : a.ny * a.nz;
  const dim3 fgrid(rows, (a.nx + 255) / 256);
  hipLaunchKernelGGL((k_adj_consfold<T, NV, MIX>), fgrid, dim3(256), 0, st, qs, P, r, a,
                     static_cast<T*>(out), mode, alpha, beta, static_cast<const T*>(y), gam,
                     zfold ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, bool HLLC, bool MIX>
int adj_rhs_t(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb, void* out,
              int mode, double alpha, double beta, const void* y, double gam, hipStream_t st) {
  int r = -1;
  switch (a.nvar) {
#define SNAP_ADJ_CASE(NVV)                                                      \
  case NVV:                                                                     \
    r = adj_rhs_nv<T, NVV, HLLC, MIX>(w, a, q, rb, out, mode, alpha, beta, y, gam, st); \
    break;
    case 5:   // the mixture needs tracers
      if constexpr (!MIX) r = adj_rhs_nv<T, 5, HLLC, false>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
      break;
    SNAP_ADJ_CASE(6)
    SNAP_ADJ_CASE(7)
    SNAP_ADJ_CASE(8)
    SNAP_ADJ_CASE(9)
    SNAP_ADJ_CASE(10)
    SNAP_ADJ_CASE(11)
    SNAP_ADJ_CASE(12)
    SNAP_ADJ_CASE(13)
#undef SNAP_ADJ_CASE
    default: r = -1;
  }
  return r;
}

}  // namespace snap
