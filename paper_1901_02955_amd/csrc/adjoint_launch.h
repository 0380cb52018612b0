// Dispatch of the adjoint kernels for one element type (included once per type).
#pragma once

#include "snap_adjoint.h"
#include "snap_internal.h"

namespace snap {

template <typename T, int NV, bool XDIR>
void adj_line_launch(const T* W, const T* r, const AdjArgs& a, int d, T* P, hipStream_t st) {
  constexpr int LN = LineShape<T, NV, XDIR>::LN, TL = LineShape<T, NV, XDIR>::TL;
  const LineGeom g = line_geom(a, d);
  const long long blocks = ((g.nlines + LN - 1) / LN) * ((g.nd + TL - 1) / TL);
  hipLaunchKernelGGL((k_adj_line<T, NV, LN, TL, XDIR>), dim3((unsigned)blocks),
                     dim3(LineTile<T, NV, LN, TL>::NTHR), 0,
                     st, W, r, a, d, P);
}

template <typename T, int NV>
int adj_rhs_nv(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb, void* out,
               int mode, double alpha, double beta, const void* y, double gam, hipStream_t st) {
  const T* qs = static_cast<const T*>(q);
  const T* r = static_cast<const T*>(rb);
  T* W = static_cast<T*>(w.W);
  T* P = static_cast<T*>(w.P);
  const int nxp = a.nx + 2 * NG, rows = (a.nz + 2 * NG) * (a.d3 ? a.ny + 2 * NG : 1);
  const dim3 pgrid(rows, (nxp + 255) / 256);
  hipLaunchKernelGGL((k_adj_prims<T, NV>), pgrid, dim3(256), 0, st, qs, a, W);
  adj_line_launch<T, NV, true>(W, r, a, 0, P, st);
  if (a.d3) adj_line_launch<T, NV, false>(W, r, a, 1, P, st);
  adj_line_launch<T, NV, false>(W, r, a, 2, P, st);
  const dim3 fgrid(a.ny * a.nz, (a.nx + 255) / 256);
  hipLaunchKernelGGL((k_adj_consfold<T, NV>), fgrid, dim3(256), 0, st, qs, P, r, a,
                     static_cast<T*>(out), mode, alpha, beta, static_cast<const T*>(y), gam);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int adj_rhs_t(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb, void* out,
              int mode, double alpha, double beta, const void* y, double gam, hipStream_t st) {
  int r = -1;
  switch (a.nvar) {
#define SNAP_ADJ_CASE(NVV)                                                      \
  case NVV:                                                                     \
    r = adj_rhs_nv<T, NVV>(w, a, q, rb, out, mode, alpha, beta, y, gam, st);   \
    break;
    SNAP_ADJ_CASE(5)
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
