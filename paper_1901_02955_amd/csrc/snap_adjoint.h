// Discrete adjoint of the right-hand side: q_bar = J(q)^T r_bar, where J is
// the Jacobian of the interior right-hand side (Sec. 4, eq. forward with the
// LMARS flux of Sec. 4.1, the WENO5 reconstruction of Sec. 4.2 and the
// conserved -> primitive map of App. B) with respect to the interior state,
// ghost cells being functions of the interior through the boundary conditions.
//
// The reverse sweep uses no atomics, so the result is reproducible bit for bit:
//   k_adj_line<d>    per direction d, per tile of lines: the primitives of
//                    the tile's cells from the state (as in the forward
//                    pass), the WENO face states recomputed, LMARS forward
//                    and reverse with the flux cotangent
//                    F_bar = (r_bar[right cell] - r_bar[left cell]) / dx_d,
//                    the WENO5 reverse to the five stencil inputs, and a
//                    fixed-order gather of those contributions into the
//                    primitive cotangent;
//   k_adj_march<d>   the same for the y and z directions in single precision,
//                    one thread per line segment marching along it; the z
//                    march also folds (below) the cells at least 3 from the
//                    y and z edges, in single precision;
//   k_adj_xmerge     before a folding z march: the x ghost cells' primitive
//                    cotangents added into the cells they copy;
//   k_adj_consfold   per interior cell (after a folding z march: the rest):
//                    gravity terms and the
//                    reverse of the conserved -> primitive map (double
//                    precision) for the cell and for each ghost cell that
//                    copies it, summed (sign flipped on the reflected normal
//                    momentum), and combined with the stage's other
//                    cotangent terms.
#pragma once

#include "snap_device.h"
#include "snap_stage.h"

namespace snap {

struct AdjArgs {
  int nx, ny, nz, gy, d3, nvar;
  long long sy, sz, sv;     // padded strides
  long long ry, rz, rv;     // interior strides
  double dxi[3];            // 1 / spacing per direction (x, y, z)
  double gamma, gm1, inv_gm1, grav, eps;
  int linear;
  int bc[3];
  int pert;   // perturbation storage (rho - rhobar_k, E - pbar_k / (gamma - 1))
  int hllc;   // the HLLC flux (else LMARS)
  int mixture;   // the mixture equation of state (App. B)
  Mixture mix;   // its coefficients
  Sediment sed;  // falling condensates (mixture only; sed.on = 0: none)
  const double* rbar_c;
  const double* pbar_c;
  const double* rbar_f;
  const double* pbar_f;
};

// Box of a per-direction work array: interior sizes with `ext` extra points
// along direction d (faces: 1, reconstructed cells: 2).
struct DirBox {
  int n[3];   // extents along x, y, z
  long long total;
};

__host__ __device__ inline DirBox dir_box(const AdjArgs& a, int d, int ext) {
  DirBox b;
  b.n[0] = a.nx + (d == 0 ? ext : 0);
  b.n[1] = a.ny + (d == 1 ? ext : 0);
  b.n[2] = a.nz + (d == 2 ? ext : 0);
  b.total = (long long)b.n[0] * b.n[1] * b.n[2];
  return b;
}

__device__ __forceinline__ void box_coords(const DirBox& b, long long g, int& x, int& y, int& z) {
  x = (int)(g % b.n[0]);
  const long long r = g / b.n[0];
  y = (int)(r % b.n[1]);
  z = (int)(r / b.n[1]);
}

__device__ __forceinline__ long long box_index(const DirBox& b, int x, int y, int z) {
  return ((long long)z * b.n[1] + y) * b.n[0] + x;
}

// padded offset of interior coordinates (i, j, k) (ghosts allowed)
__device__ __forceinline__ long long padded_off(const AdjArgs& a, int i, int j, int k) {
  return (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
}

// ---------------------------------------------------------------------------
// WENO5 of one cell split for the reverse sweep (same formulation as
// weno5_cell). weno5_lin returns both face values and keeps the forward
// quantities the linearisation needs; weno5_rev maps the cotangents gm of qm
// and gp of qp back to the five inputs a..e.
// As in weno5_cell the smoothness sums are formed as 4 s_k = 4 eps + (13/3)
// u_k^2 + v_k^2 (the normalised weights depend only on their ratios), and
// they are scaled by a common power of two (exact) so that the products of
// squared sums below stay in range in single precision.
// ---------------------------------------------------------------------------
template <typename T>
struct WenoLin {
  T s0, s1, s2, sc;                // scaled smoothness sums, and the scale
  T wm0, wm1, wm2, wp0, wp1, wp2;  // normalised weights of qm and of qp
  T idm, idp;                      // reciprocals of the unnormalised weight sums
};

template <typename T>
__device__ __forceinline__ void weno5_lin(T a, T b, T c, T d, T e, T eps, bool linear,
                                          WenoLin<T>& L, T& qm, T& qp) {
  const T da = a - c, db = b - c, dd = d - c, de = e - c;
  const T m0 = T(2) * da - T(7) * db, m1 = T(2) * dd - db, m2 = T(5) * dd - de;
  const T p0 = T(2) * de - T(7) * dd, p1 = T(2) * db - dd, p2 = T(5) * db - da;
  const T sixth = T(1) / T(6);
  if (linear) {
    qm = c + (T(0.1) * m0 + T(0.6) * m1 + T(0.3) * m2) * sixth;
    qp = c + (T(0.1) * p0 + T(0.6) * p1 + T(0.3) * p2) * sixth;
    return;
  }
  const T k13 = T(13) / T(3), eps4 = T(4) * eps;
  const T u0 = fma(T(-2), db, da), v0 = fma(T(-4), db, da);
  const T u1 = db + dd, v1 = db - dd;
  const T u2 = fma(T(-2), dd, de), v2 = fma(T(-4), dd, de);
  T s0 = fma(v0, v0, fma(k13 * u0, u0, eps4));
  T s1 = fma(v1, v1, fma(k13 * u1, u1, eps4));
  T s2 = fma(v2, v2, fma(k13 * u2, u2, eps4));
  T sc;
  if constexpr (sizeof(T) == 4) {
    const float mx = fmaxf(fmaxf(s0, s1), s2);
    sc = __builtin_amdgcn_ldexpf(1.0f, -__builtin_amdgcn_frexp_expf(mx));
  } else {
    const double mx = fmax(fmax(s0, s1), s2);
    sc = __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(mx));
  }
  s0 *= sc;
  s1 *= sc;
  s2 *= sc;
  const T q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
  const T t0 = q1 * q2, t1 = q0 * q2, t2 = q0 * q1;
  const T n0 = T(0.1) * t0, n1 = T(0.6) * t1, n2 = T(0.3) * t2;
  const T r0 = T(0.1) * t2, r1 = T(0.6) * t1, r2 = T(0.3) * t0;
  const T idm = rcp_fast(n0 + n1 + n2), idp = rcp_fast(r0 + r1 + r2);
  L.s0 = s0;
  L.s1 = s1;
  L.s2 = s2;
  L.sc = sc;
  L.wm0 = n0 * idm;
  L.wm1 = n1 * idm;
  L.wm2 = n2 * idm;
  L.wp0 = r0 * idp;
  L.wp1 = r1 * idp;
  L.wp2 = r2 * idp;
  L.idm = idm;
  L.idp = idp;
  qm = c + (L.wm0 * m0 + L.wm1 * m1 + L.wm2 * m2) * sixth;
  qp = c + (L.wp0 * p0 + L.wp1 * p1 + L.wp2 * p2) * sixth;
}

template <typename T>
__device__ __forceinline__ void weno5_rev(T a, T b, T c, T d, T e, bool linear,
                                          const WenoLin<T>& L, T gm, T gp, T (&g)[5]) {
  const T da = a - c, db = b - c, dd = d - c, de = e - c;
  const T sixth = T(1) / T(6);
  T mb0, mb1, mb2, pb0, pb1, pb2;
  T ub0 = T(0), vb0 = T(0), ub1 = T(0), vb1 = T(0), ub2 = T(0), vb2 = T(0);
  if (linear) {
    mb0 = gm * T(0.1) * sixth;
    mb1 = gm * T(0.6) * sixth;
    mb2 = gm * T(0.3) * sixth;
    pb0 = gp * T(0.1) * sixth;
    pb1 = gp * T(0.6) * sixth;
    pb2 = gp * T(0.3) * sixth;
  } else {
    const T m0 = T(2) * da - T(7) * db, m1 = T(2) * dd - db, m2 = T(5) * dd - de;
    const T p0 = T(2) * de - T(7) * dd, p1 = T(2) * db - dd, p2 = T(5) * db - da;
    const T Mm = L.wm0 * m0 + L.wm1 * m1 + L.wm2 * m2;   // 6 (qm - c)
    const T Mp = L.wp0 * p0 + L.wp1 * p1 + L.wp2 * p2;
    const T gms = gm * sixth, gps = gp * sixth;
    mb0 = gms * L.wm0;
    mb1 = gms * L.wm1;
    mb2 = gms * L.wm2;
    pb0 = gps * L.wp0;
    pb1 = gps * L.wp1;
    pb2 = gps * L.wp2;
    // cotangents of the unnormalised weights
    const T gmD = gms * L.idm, gpD = gps * L.idp;
    const T nb0 = gmD * (m0 - Mm), nb1 = gmD * (m1 - Mm), nb2 = gmD * (m2 - Mm);
    const T rb0 = gpD * (p0 - Mp), rb1 = gpD * (p1 - Mp), rb2 = gpD * (p2 - Mp);
    const T tb0 = T(0.1) * nb0 + T(0.3) * rb2;
    const T tb1 = T(0.6) * (nb1 + rb1);
    const T tb2 = T(0.3) * nb2 + T(0.1) * rb0;
    const T q0 = L.s0 * L.s0, q1 = L.s1 * L.s1, q2 = L.s2 * L.s2;
    const T qb0 = tb1 * q2 + tb2 * q1;
    const T qb1 = tb0 * q2 + tb2 * q0;
    const T qb2 = tb0 * q1 + tb1 * q0;
    // cotangent of the unscaled 4 s_k: sc * 2 s'_k * qb_k (s'_k the scaled
    // sum kept by the forward), times d(4 s)/du = (26/3) u and d(4 s)/dv = 2 v
    const T two_sc = T(2) * L.sc;
    const T bb0 = two_sc * L.s0 * qb0;
    const T bb1 = two_sc * L.s1 * qb1;
    const T bb2 = two_sc * L.s2 * qb2;
    const T k263 = T(26) / T(3);
    ub0 = k263 * fma(T(-2), db, da) * bb0;
    vb0 = T(2) * fma(T(-4), db, da) * bb0;
    ub1 = k263 * (db + dd) * bb1;
    vb1 = T(2) * (db - dd) * bb1;
    ub2 = k263 * fma(T(-2), dd, de) * bb2;
    vb2 = T(2) * fma(T(-4), dd, de) * bb2;
  }
  const T dab = T(2) * mb0 - pb2 + ub0 + vb0;
  const T dbb = -T(7) * mb0 - mb1 + T(2) * pb1 + T(5) * pb2 - T(2) * ub0 - T(4) * vb0 + ub1 + vb1;
  const T ddb = T(2) * mb1 + T(5) * mb2 - T(7) * pb0 - pb1 + ub1 - vb1 - T(2) * ub2 - T(4) * vb2;
  const T deb = -mb2 + T(2) * pb0 + ub2 + vb2;
  g[0] = dab;
  g[1] = dbb;
  g[2] = gm + gp - (dab + dbb + ddb + deb);
  g[3] = ddb;
  g[4] = deb;
}

// ---------------------------------------------------------------------------
// Forward and reverse of one WENO5 cell in one pass: the cotangents g of the
// five inputs a..e given the cotangents gm of qm and gp of qp (the transpose
// of the derivative of weno5_cell at a..e), for a caller that does not keep
// the forward quantities. With S_k = 4 eps + (13/3) u_k^2 + v_k^2 and the
// normalised weights w_k = (d_k / S_k^2) / sum_m (d_m / S_m^2), the derivative
// of qm - c = (1/6) sum_k w_k m_k with respect to S_j is
// -(w_j / (3 S_j)) (m_j - M) with M = sum_k w_k m_k, and qp's stencil k uses
// S_{2-k}. Hence the cotangent of S_j is
//   Sb_j = -2 (mb_j (m_j - Mm) + pb_{2-j} (p_{2-j} - Mp)) / S_j,
// where mb_k = gm w_k / 6 and pb_k = gp wp_k / 6 are the cotangents of the
// candidate values, and those of u_j and v_j are Sb_j (26/3) u_j and Sb_j 2 v_j
// (dS/du = (26/3) u, dS/dv = 2 v). The weights are formed as in weno5_lin.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void weno5_linrev(T a, T b, T c, T d, T e, T eps, bool linear, T gm,
                                             T gp, T (&g)[5]) {
  const T da = a - c, db = b - c, dd = d - c, de = e - c;
  const T sixth = T(1) / T(6);
  const T gms = gm * sixth, gps = gp * sixth;
  T mb0, mb1, mb2, pb0, pb1, pb2;
  T ub0 = T(0), vb0 = T(0), ub1 = T(0), vb1 = T(0), ub2 = T(0), vb2 = T(0);
  if (linear) {
    mb0 = gms * T(0.1);
    mb1 = gms * T(0.6);
    mb2 = gms * T(0.3);
    pb0 = gps * T(0.1);
    pb1 = gps * T(0.6);
    pb2 = gps * T(0.3);
  } else {
    const T m0 = T(2) * da - T(7) * db, m1 = T(2) * dd - db, m2 = T(5) * dd - de;
    const T p0 = T(2) * de - T(7) * dd, p1 = T(2) * db - dd, p2 = T(5) * db - da;
    const T k13 = T(13) / T(3), eps4 = T(4) * eps;
    const T u0 = fma(T(-2), db, da), v0 = fma(T(-4), db, da);
    const T u1 = db + dd, v1 = db - dd;
    const T u2 = fma(T(-2), dd, de), v2 = fma(T(-4), dd, de);
    const T ku0 = k13 * u0, ku1 = k13 * u1, ku2 = k13 * u2;
    const T S0 = fma(v0, v0, fma(ku0, u0, eps4));
    const T S1 = fma(v1, v1, fma(ku1, u1, eps4));
    const T S2 = fma(v2, v2, fma(ku2, u2, eps4));
    T sc;
    if constexpr (sizeof(T) == 4) {
      // 2^-E, E the exponent of the largest sum (from its exponent bits)
      const float mx = fmaxf(fmaxf(S0, S1), S2);
      sc = __uint_as_float(0x7F000000u - (__float_as_uint(mx) & 0x7F800000u));
    } else {
      const double mx = fmax(fmax(S0, S1), S2);
      sc = __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(mx));
    }
    const T s0 = S0 * sc, s1 = S1 * sc, s2 = S2 * sc;
    const T q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
    const T t0 = q1 * q2, t1 = q0 * q2, t2 = q0 * q1;
    // unnormalised weights (the middle one is the same for both faces)
    const T n0 = T(0.1) * t0, n1 = T(0.6) * t1, n2 = T(0.3) * t2;
    const T r0 = T(0.1) * t2, r2 = T(0.3) * t0;
    const T idm = rcp_fast(n0 + n1 + n2), idp = rcp_fast(r0 + n1 + r2);
    // M = sum_k w_k m_k = idm sum_k n_k m_k, and mb_k = gm w_k / 6
    const T Mm = idm * fma(n0, m0, fma(n1, m1, n2 * m2));
    const T Mp = idp * fma(r0, p0, fma(n1, p1, r2 * p2));
    const T gmw = gms * idm, gpw = gps * idp;
    mb0 = gmw * n0;
    mb1 = gmw * n1;
    mb2 = gmw * n2;
    pb0 = gpw * r0;
    pb1 = gpw * n1;
    pb2 = gpw * r2;
    // h_j = 2 Sb_j, so that ub_j = h_j (13/3) u_j and vb_j = h_j v_j
    const T h0 = T(-4) * fma(mb0, m0 - Mm, pb2 * (p2 - Mp)) * rcp_fast(S0);
    const T h1 = T(-4) * fma(mb1, m1 - Mm, pb1 * (p1 - Mp)) * rcp_fast(S1);
    const T h2 = T(-4) * fma(mb2, m2 - Mm, pb0 * (p0 - Mp)) * rcp_fast(S2);
    ub0 = h0 * ku0;
    vb0 = h0 * v0;
    ub1 = h1 * ku1;
    vb1 = h1 * v1;
    ub2 = h2 * ku2;
    vb2 = h2 * v2;
  }
  const T dab = T(2) * mb0 - pb2 + ub0 + vb0;
  const T dbb = -T(7) * mb0 - mb1 + T(2) * pb1 + T(5) * pb2 - T(2) * ub0 - T(4) * vb0 + ub1 + vb1;
  const T ddb = T(2) * mb1 + T(5) * mb2 - T(7) * pb0 - pb1 + ub1 - vb1 - T(2) * ub2 - T(4) * vb2;
  const T deb = -mb2 + T(2) * pb0 + ub2 + vb2;
  g[0] = dab;
  g[1] = dbb;
  g[2] = gm + gp - (dab + dbb + ddb + deb);
  g[3] = ddb;
  g[4] = deb;
}

// ---------------------------------------------------------------------------
// Reverse of lmars_flux: given the flux cotangent fb, accumulate the
// cotangents of the two face states into xlb / xrb. At u* == 0 the derivative
// of the advective flux with respect to u* uses the mean of both sides'
// advected vectors.
// ---------------------------------------------------------------------------
template <typename T, int NV>
__device__ __forceinline__ void lmars_flux_adj(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                               T rref, T pref, T gamma, T inv_gm1,
                                               const T (&fb)[NV], T (&xlb)[NV], T (&xrb)[NV]) {
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  const T unl = xl[nrm], unr = xr[nrm];
  T hl, hr;   // 1 / sqrt(gamma p rho) of each side
  const T cl = sound_speed_h(gamma * pl, rl, hl), cr = sound_speed_h(gamma * pr, rr, hr);
  const T ra = T(0.5) * (rl + rr), ca = T(0.5) * (cl + cr);
  const T rc = ra * ca;
  const T hh = T(0.5) * rcp_fast(rc);
  const T ustar = T(0.5) * (unl + unr) - (xr[4] - xl[4]) * hh;
  // advected vectors of both sides
  auto adv = [&](const T (&x)[NV], T r, T p, T (&phi)[NV]) {
    const T k = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    phi[0] = r;
    phi[1] = r * x[1];
    phi[2] = r * x[2];
    phi[3] = r * x[3];
    phi[4] = p * inv_gm1 + r * k + p;
#pragma unroll
    for (int t = 5; t < NV; ++t) phi[t] = r * x[t];
  };
  T phl[NV], phr[NV];
  adv(xl, rl, pl, phl);
  adv(xr, rr, pr, phr);
  T usb = T(0);
  const T wl = ustar > T(0) ? T(1) : (ustar < T(0) ? T(0) : T(0.5));
#pragma unroll
  for (int m = 0; m < NV; ++m) usb += fb[m] * (wl * phl[m] + (T(1) - wl) * phr[m]);
  const T psb = fb[nrm];
  // advected-vector cotangents of the upwind side (zero at u* == 0); the side
  // is selected element by element so that both state arrays stay in registers
  {
    const bool left = ustar > T(0);
    T x[NV], phb[NV], sb[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      x[m] = left ? xl[m] : xr[m];
      phb[m] = ustar * fb[m];
    }
    const T r = left ? rl : rr;
    const T k = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    T rbs = phb[0] + phb[1] * x[1] + phb[2] * x[2] + phb[3] * x[3] + phb[4] * k;
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      rbs += phb[t] * x[t];
      sb[t] = phb[t] * r;
    }
    sb[0] = rbs;
    sb[1] = phb[1] * r + phb[4] * r * x[1];
    sb[2] = phb[2] * r + phb[4] * r * x[2];
    sb[3] = phb[3] * r + phb[4] * r * x[3];
    sb[4] = phb[4] * (inv_gm1 + T(1));
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      xlb[m] += left ? sb[m] : T(0);
      xrb[m] += left ? T(0) : sb[m];
    }
  }
  // u* = (unl + unr)/2 - (p'_R - p'_L) hh,  hh = 1 / (2 rc)
  T rcb = T(0);
  xlb[nrm] += T(0.5) * usb;
  xrb[nrm] += T(0.5) * usb;
  xrb[4] -= usb * hh;
  xlb[4] += usb * hh;
  rcb += -usb * (xr[4] - xl[4]) * (-T(2) * hh * hh);
  // p* = (p'_L + p'_R)/2 - rc (unr - unl)/2
  xlb[4] += T(0.5) * psb;
  xrb[4] += T(0.5) * psb;
  rcb += -T(0.5) * (unr - unl) * psb;
  xrb[nrm] += -T(0.5) * rc * psb;
  xlb[nrm] += T(0.5) * rc * psb;
  // rc = ra ca
  const T rab = rcb * ca, cab = rcb * ra;
  T rlb = T(0.5) * rab, rrb = T(0.5) * rab;
  const T clb = T(0.5) * cab, crb = T(0.5) * cab;
  // c = gamma p h with h = 1 / sqrt(gamma p rho) = 1 / (rho c):
  // dc/dp = gamma / (2 rho c) = gamma h / 2, dc/drho = -c / (2 rho) = -c^2 h / 2
  const T hcl = T(0.5) * clb * hl, hcr = T(0.5) * crb * hr;
  xlb[4] += hcl * gamma;
  rlb += -hcl * cl * cl;
  xrb[4] += hcr * gamma;
  rrb += -hcr * cr * cr;
  xlb[0] += rlb;
  xrb[0] += rrb;
}

// ---------------------------------------------------------------------------
// Reverse of hllc_flux: given the flux cotangent fb, accumulate the
// cotangents of the two face states into xlb / xrb. The branch (the side k
// whose flux is taken, and whether the star correction applies) is that of
// the forward evaluation; the outer speeds take the derivative of the
// candidate that min / max selected. With c = sqrt(gamma p / rho):
// dc/dp = c / (2 p), dc/drho = -c / (2 rho).
// ---------------------------------------------------------------------------
template <typename T, int NV>
__device__ __forceinline__ void hllc_flux_adj(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                              T rref, T pref, T gamma, T inv_gm1,
                                              const T (&fb)[NV], T (&xlb)[NV], T (&xrb)[NV]) {
  // ---- forward, as in hllc_flux
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  const T unl = nrm == 1 ? xl[1] : (nrm == 2 ? xl[2] : xl[3]);
  const T unr = nrm == 1 ? xr[1] : (nrm == 2 ? xr[2] : xr[3]);
  const T cl = sound_speed(gamma * pl, rl);
  const T cr = sound_speed(gamma * pr, rr);
  const bool sl_left = unl - cl <= unr - cr, sr_left = unl + cl >= unr + cr;
  const T SL = sl_left ? unl - cl : unr - cr, SR = sr_left ? unl + cl : unr + cr;
  const T dl = rl * (SL - unl), dr = rr * (SR - unr);
  const T iD = rcp_fast(dl - dr);
  const T Ss = (pr - pl + dl * unl - dr * unr) * iD;
  const bool left = SL >= T(0) || Ss >= T(0);
  const bool star = !(SL >= T(0)) && (left || SR > T(0));
  const T rk = left ? rl : rr, pk = left ? pl : pr;
  T vk[3];
  vk[0] = left ? xl[1] : xr[1];
  vk[1] = left ? xl[2] : xr[2];
  vk[2] = left ? xl[3] : xr[3];
  const T unk = left ? unl : unr, Sk = left ? SL : SR, dk = left ? dl : dr;
  const T E = pk * inv_gm1 + T(0.5) * rk * (vk[0] * vk[0] + vk[1] * vk[1] + vk[2] * vk[2]);
  const T mass = rk * unk;
  // ---- reverse: cotangents of the side quantities
  T rkb = T(0), pkb = T(0), ppkb = T(0), unkb = T(0), Skb = T(0), dkb = T(0), Ssb = T(0);
  T Eb = T(0), massb = T(0);
  T vb[3] = {T(0), T(0), T(0)};
  T qb[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) qb[t] = T(0);
  if (star) {
    const T W = Sk - Ss, iW = rcp_fast(W);
    const T fac = dk * iW;
    const T idk = rcp_fast(dk), irk = rcp_fast(rk);
    const T A1 = Ss - unk, A2 = Ss + pk * idk;
    const T B = E * irk + A1 * A2;
    const T e_star = fac * B;
    T facb = T(0);
    // f0 += Sk (fac - rk)
    Skb += fb[0] * (fac - rk);
    facb += fb[0] * Sk;
    rkb -= fb[0] * Sk;
    // f_i += Sk (fac s_i - rk u_i), s_i = S* on the normal, else u_i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T g = fb[1 + i];
      const bool nn = (i + 1) == nrm;
      const T si = nn ? Ss : vk[i];
      Skb += g * (fac * si - rk * vk[i]);
      facb += g * Sk * si;
      if (nn)
        Ssb += g * Sk * fac;
      else
        vb[i] += g * Sk * fac;
      rkb -= g * Sk * vk[i];
      vb[i] -= g * Sk * rk;
    }
    // f4 += Sk (e_star - E)
    Skb += fb[4] * (e_star - E);
    const T esb = fb[4] * Sk;
    Eb -= fb[4] * Sk;
    // f_t += Sk (fac - rk) q_t
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      const T qk = left ? xl[t] : xr[t];
      Skb += fb[t] * (fac - rk) * qk;
      facb += fb[t] * Sk * qk;
      rkb -= fb[t] * Sk * qk;
      qb[t] += fb[t] * Sk * (fac - rk);
    }
    // e_star = fac B, B = E / rk + (S* - un)(S* + p / dk)
    facb += esb * B;
    const T Bb = esb * fac;
    Eb += Bb * irk;
    rkb -= Bb * E * irk * irk;
    Ssb += Bb * (A1 + A2);
    unkb -= Bb * A2;
    pkb += Bb * A1 * idk;
    dkb -= Bb * A1 * pk * idk * idk;
    // fac = dk / (Sk - S*)
    dkb += facb * iW;
    const T Wb = -facb * fac * iW;
    Skb += Wb;
    Ssb -= Wb;
  }
  // plain flux of side k: f0 = mass, f_i = mass u_i (+ p' on the normal),
  // f4 = (E + p) un, f_t = mass q_t
  massb += fb[0];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    massb += fb[1 + i] * vk[i];
    vb[i] += fb[1 + i] * mass;
  }
  ppkb += nrm == 1 ? fb[1] : (nrm == 2 ? fb[2] : fb[3]);
  Eb += fb[4] * unk;
  pkb += fb[4] * unk;
  unkb += fb[4] * (E + pk);
#pragma unroll
  for (int t = 5; t < NV; ++t) {
    const T qk = left ? xl[t] : xr[t];
    massb += fb[t] * qk;
    qb[t] += fb[t] * mass;
  }
  rkb += massb * unk;
  unkb += massb * rk;
  pkb += Eb * inv_gm1;
  rkb += Eb * T(0.5) * (vk[0] * vk[0] + vk[1] * vk[1] + vk[2] * vk[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) vb[i] += Eb * rk * vk[i];
  // the normal velocity of side k is one of its velocities
  vb[nrm - 1] += unkb;
  // ---- back to both sides: S* = N / D, N = pr - pl + dl unl - dr unr, D = dl - dr
  T rlb = T(0), rrb = T(0), plb = T(0), prb = T(0), unlb = T(0), unrb = T(0);
  T dlb = left ? dkb : T(0), drb = left ? T(0) : dkb;
  T SLb = left ? Skb : T(0), SRb = left ? T(0) : Skb;
  {
    const T Nb = Ssb * iD, Db = -Ssb * Ss * iD;
    prb += Nb;
    plb -= Nb;
    dlb += Nb * unl + Db;
    unlb += Nb * dl;
    drb += -Nb * unr - Db;
    unrb -= Nb * dr;
  }
  // dl = rl (SL - unl), dr = rr (SR - unr)
  rlb += dlb * (SL - unl);
  SLb += dlb * rl;
  unlb -= dlb * rl;
  rrb += drb * (SR - unr);
  SRb += drb * rr;
  unrb -= drb * rr;
  // SL = min(unl - cl, unr - cr), SR = max(unl + cl, unr + cr)
  T clb = T(0), crb = T(0);
  if (sl_left) {
    unlb += SLb;
    clb -= SLb;
  } else {
    unrb += SLb;
    crb -= SLb;
  }
  if (sr_left) {
    unlb += SRb;
    clb += SRb;
  } else {
    unrb += SRb;
    crb += SRb;
  }
  plb += clb * cl * T(0.5) * rcp_fast(pl);
  rlb -= clb * cl * T(0.5) * rcp_fast(rl);
  prb += crb * cr * T(0.5) * rcp_fast(pr);
  rrb -= crb * cr * T(0.5) * rcp_fast(rr);
  // side k's own quantities: rho = rref + x0, p = pref + x4, p' = x4
  if (left) {
    rlb += rkb;
    plb += pkb + ppkb;
  } else {
    rrb += rkb;
    prb += pkb + ppkb;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    xlb[1 + i] += left ? vb[i] : T(0);
    xrb[1 + i] += left ? T(0) : vb[i];
  }
#pragma unroll
  for (int t = 5; t < NV; ++t) {
    xlb[t] += left ? qb[t] : T(0);
    xrb[t] += left ? T(0) : qb[t];
  }
  // the normal velocities of both sides enter the wave speeds
  xlb[nrm] += unlb;
  xrb[nrm] += unrb;
  xlb[0] += rlb;
  xrb[0] += rrb;
  xlb[4] += plb;
  xrb[4] += prb;
}

// ---------------------------------------------------------------------------
// Reverse of lmars_flux_mix (the mixture equation of state): as
// lmars_flux_adj, plus the sums n = 1 + sum a_t q_t, d = 1 + sum b_t q_t and
// m = sum mu_t q_t of each side's face mass fractions, which enter its sound
// speed c = sqrt((d + gm1 n) p / (d rho)) and the upwind side's energy
// E = p d / (gm1 n) + rho (|u|^2 / 2 + m). At u* == 0 the derivative with
// respect to u* uses the mean of both sides' advected vectors.
// ---------------------------------------------------------------------------
template <typename T, int NV>
__device__ __forceinline__ void lmars_flux_mix_adj(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                                   T rref, T pref, T gm1, const Mixture& mx,
                                                   const T (&fb)[NV], T (&xlb)[NV],
                                                   T (&xrb)[NV]) {
  constexpr int NT = NV - 5;
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  const T unl = nrm == 1 ? xl[1] : (nrm == 2 ? xl[2] : xl[3]);
  const T unr = nrm == 1 ? xr[1] : (nrm == 2 ? xr[2] : xr[3]);
  T nl = T(1), dl = T(1), ml = T(0), nr = T(1), dr = T(1), mr = T(0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T at, bt, mt;
    mixture_coef<T, NT>(mx, t, at, bt, mt);
    nl += at * xl[5 + t];
    dl += bt * xl[5 + t];
    ml += mt * xl[5 + t];
    nr += at * xr[5 + t];
    dr += bt * xr[5 + t];
    mr += mt * xr[5 + t];
  }
  const T gnl = gm1 * nl, gnr = gm1 * nr;
  const T cl = sound_speed((dl + gnl) * pl, dl * rl);
  const T cr = sound_speed((dr + gnr) * pr, dr * rr);
  const T rc = T(0.25) * ((rl + rr) * (cl + cr));
  const T hh = T(0.5) * rcp_fast(rc);
  const T ustar = T(0.5) * (unl + unr) - (xr[4] - xl[4]) * hh;
  // advected vectors (rho, rho u, rho v, rho w, E + p, rho q) of both sides
  auto adv = [&](const T (&x)[NV], T r, T p, T d, T gn, T m, T (&phi)[NV]) {
    const T k = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    phi[0] = r;
    phi[1] = r * x[1];
    phi[2] = r * x[2];
    phi[3] = r * x[3];
    phi[4] = p * d * rcp_fast(gn) + r * (k + m) + p;
#pragma unroll
    for (int t = 5; t < NV; ++t) phi[t] = r * x[t];
  };
  T phl[NV], phr[NV];
  adv(xl, rl, pl, dl, gnl, ml, phl);
  adv(xr, rr, pr, dr, gnr, mr, phr);
  const T wl = ustar > T(0) ? T(1) : (ustar < T(0) ? T(0) : T(0.5));
  T usb = T(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) usb += fb[v] * (wl * phl[v] + (T(1) - wl) * phr[v]);
  const T psb = fb[nrm];
  // cotangents of each side's rho, p, n, d, m (the velocities and fractions go
  // straight into xlb / xrb)
  T rlb = T(0), rrb = T(0), plb = T(0), prb = T(0);
  T nlb = T(0), nrb = T(0), dlb = T(0), drb = T(0), mlb = T(0), mrb = T(0);
  {
    const bool left = ustar > T(0);
    const T r = left ? rl : rr, p = left ? pl : pr, d = left ? dl : dr;
    const T gn = left ? gnl : gnr, m = left ? ml : mr;
    T x[NV], phb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      x[v] = left ? xl[v] : xr[v];
      phb[v] = ustar * fb[v];
    }
    const T k = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    const T ign = rcp_fast(gn);
    // phi4 = p d / gn + r (k + m) + p
    T rb_ = phb[0] + phb[1] * x[1] + phb[2] * x[2] + phb[3] * x[3] + phb[4] * (k + m);
    const T pb_ = phb[4] * (d * ign + T(1));
    const T db_ = phb[4] * p * ign;
    const T gnb = -phb[4] * p * d * ign * ign;
    const T mb_ = phb[4] * r;
    T sb[NV];
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      rb_ += phb[t] * x[t];
      sb[t] = phb[t] * r;
    }
    sb[0] = T(0);
    sb[4] = T(0);
    sb[1] = phb[1] * r + phb[4] * r * x[1];
    sb[2] = phb[2] * r + phb[4] * r * x[2];
    sb[3] = phb[3] * r + phb[4] * r * x[3];
#pragma unroll
    for (int v = 1; v < NV; ++v) {
      if (v == 4) continue;
      xlb[v] += left ? sb[v] : T(0);
      xrb[v] += left ? T(0) : sb[v];
    }
    rlb += left ? rb_ : T(0);
    rrb += left ? T(0) : rb_;
    plb += left ? pb_ : T(0);
    prb += left ? T(0) : pb_;
    dlb += left ? db_ : T(0);
    drb += left ? T(0) : db_;
    nlb += left ? gm1 * gnb : T(0);
    nrb += left ? T(0) : gm1 * gnb;
    mlb += left ? mb_ : T(0);
    mrb += left ? T(0) : mb_;
  }
  // u* = (unl + unr) / 2 - (p'_R - p'_L) hh, hh = 1 / (2 rc)
  T rcb = usb * (xr[4] - xl[4]) * (T(2) * hh * hh);
  xlb[nrm] += T(0.5) * usb;
  xrb[nrm] += T(0.5) * usb;
  xrb[4] -= usb * hh;
  xlb[4] += usb * hh;
  // p* = (p'_L + p'_R) / 2 - rc (unr - unl) / 2
  xlb[4] += T(0.5) * psb;
  xrb[4] += T(0.5) * psb;
  rcb -= T(0.5) * (unr - unl) * psb;
  xrb[nrm] -= T(0.5) * rc * psb;
  xlb[nrm] += T(0.5) * rc * psb;
  // rc = (rl + rr)(cl + cr) / 4
  rlb += T(0.25) * rcb * (cl + cr);
  rrb += T(0.25) * rcb * (cl + cr);
  const T clb = T(0.25) * rcb * (rl + rr), crb = T(0.25) * rcb * (rl + rr);
  // c = sqrt(G / R), G = (d + gm1 n) p, R = d rho: dc/dG = c / (2 G), dc/dR = -c / (2 R)
  {
    const T G = (dl + gnl) * pl, R = dl * rl;
    const T Gb = clb * cl * T(0.5) * rcp_fast(G), Rb = -clb * cl * T(0.5) * rcp_fast(R);
    dlb += Gb * pl + Rb * rl;
    nlb += Gb * pl * gm1;
    plb += Gb * (dl + gnl);
    rlb += Rb * dl;
  }
  {
    const T G = (dr + gnr) * pr, R = dr * rr;
    const T Gb = crb * cr * T(0.5) * rcp_fast(G), Rb = -crb * cr * T(0.5) * rcp_fast(R);
    drb += Gb * pr + Rb * rr;
    nrb += Gb * pr * gm1;
    prb += Gb * (dr + gnr);
    rrb += Rb * dr;
  }
  // n, d, m are linear in the fractions
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T at, bt, mt;
    mixture_coef<T, NT>(mx, t, at, bt, mt);
    xlb[5 + t] += at * nlb + bt * dlb + mt * mlb;
    xrb[5 + t] += at * nrb + bt * drb + mt * mrb;
  }
  xlb[0] += rlb;
  xrb[0] += rrb;
  xlb[4] += plb;
  xrb[4] += prb;
}

// Reverse of the kernel's Riemann flux (LMARS, HLLC, or LMARS under the
// mixture equation of state).
template <typename T, int NV, bool HLLC, bool MIX>
__device__ __forceinline__ void riemann_flux_adj(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                                 T rref, T pref, T gamma, T inv_gm1, T gm1,
                                                 const Mixture& mx, const T (&fb)[NV],
                                                 T (&xlb)[NV], T (&xrb)[NV]) {
  static_assert(!(HLLC && MIX), "HLLC takes passive tracers");
  if constexpr (HLLC)
    hllc_flux_adj<T, NV>(xl, xr, nrm, rref, pref, gamma, inv_gm1, fb, xlb, xrb);
  else if constexpr (MIX)
    lmars_flux_mix_adj<T, NV>(xl, xr, nrm, rref, pref, gm1, mx, fb, xlb, xrb);
  else
    lmars_flux_adj<T, NV>(xl, xr, nrm, rref, pref, gamma, inv_gm1, fb, xlb, xrb);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Fused adjoint of one direction d for a tile of LN lines x TL cells along d.
// In LDS: (A) left/right face states of the reconstructed cells the tile
// needs, (B) LMARS forward and reverse at its faces with the flux cotangent
// from r_bar, (C) WENO5 reverse of its reconstructed cells (the cotangents of
// their five inputs), (D) for every cell of the tile (and the ghost cells
// beyond a domain edge) the fixed-order sum of the contributions that reach
// it, added into the primitive cotangent P. Deterministic: every sum has one
// fixed order and the directions run as separate launches.
// ---------------------------------------------------------------------------
template <typename T, int NV, int LN, int TL>
struct LineTile {
  static constexpr int NA = TL + 6;   // reconstructed cells -3 .. TL+2 (relative)
  static constexpr int NF = TL + 5;   // faces -2 .. TL+2
  static constexpr int NC = TL + 4;   // reverse-reconstructed cells -2 .. TL+1
  // threads: the largest phase (NA items per line) in one round of whole waves
  static constexpr int NTHR = (LN * NA + 63) / 64 * 64;
  // the face states are dead once (B) has read them: (C) writes over them
  union {
    struct {
      T QM[NV][LN][NA];   // left state at face j+1 of reconstructed cell j
      T QP[NV][LN][NA];   // right state at face j
    };
    T C[5][NV][LN][NC];   // cotangents of the five inputs of reconstructed cell j
  };
  T XL[NV][LN][NF];   // cotangent of the left state at face f
  T XR[NV][LN][NF];   // cotangent of the right state at face f
  T WL[NV][LN][TL + 10];   // primitives of cells -5 .. TL+4 (relative), the stencils of (A) and (C)
  long long pbase[LN];  // padded offset of position 0 of each line
  long long rbase[LN];  // interior offset of position 0 of each line
  int lev[LN];          // level (z index) of each line (x and y lines)
};

// Tile shape per element type, variable count and direction (x lines are
// contiguous; y and z lines are consecutive in x): 3 x lines of 64 cells and
// 8 y / z lines of 16 cells, or shorter lines where that tile would exceed
// 64 KiB of LDS. Small tiles let four to six workgroups share a compute unit;
// on the single-precision 256 x 256 x 128 right-hand-side adjoint they took
// 1.61 ms against 2.17 ms for 4 x 64 and 8 x 32 cells, the halo work they add
// notwithstanding. Three x lines rather than two put 210 of the (A)-phase
// items on 256 threads instead of 140 on 192 (1.47 -> 1.40 ms; 4 x 32, 5 x 32,
// 6 x 32, 10 x 32 and 4 x 64 measured slower or even).
#ifndef SNAP_ADJ_XLN
#define SNAP_ADJ_XLN 3
#endif
#ifndef SNAP_ADJ_XTL
#define SNAP_ADJ_XTL 64
#endif
#ifndef SNAP_ADJ_YLN
#define SNAP_ADJ_YLN 8
#endif
#ifndef SNAP_ADJ_YTL
#define SNAP_ADJ_YTL 16
#endif
template <typename T, int NV, bool XDIR>
struct LineShape {
  static constexpr int L0 = XDIR ? SNAP_ADJ_XLN : SNAP_ADJ_YLN;
  static constexpr int T0 = XDIR ? SNAP_ADJ_XTL : SNAP_ADJ_YTL;
  static constexpr bool A = sizeof(LineTile<T, NV, L0, T0>) <= 65536;
  static constexpr bool B = sizeof(LineTile<T, NV, L0, T0 / 2>) <= 65536;
  static constexpr int LN = A || B ? L0 : (L0 + 1) / 2;
  static constexpr int TL = A ? T0 : T0 / 2;
};

struct LineGeom {
  int d;          // direction
  int nd;         // cells along d
  long long nlines;
  long long sd;   // padded stride along d
  long long rd;   // interior stride along d
};

__host__ __device__ inline LineGeom line_geom(const AdjArgs& a, int d) {
  LineGeom g;
  g.d = d;
  g.nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
  g.nlines = d == 0 ? (long long)a.ny * a.nz : (d == 1 ? (long long)a.nx * a.nz : (long long)a.nx * a.ny);
  g.sd = d == 0 ? 1 : (d == 1 ? a.sy : a.sz);
  g.rd = d == 0 ? 1 : (d == 1 ? a.ry : a.rz);
  return g;
}

// interior coordinates (i, j, k) of position p on line L of direction d;
// lines are numbered with the lower transverse axis fastest
__device__ __forceinline__ void line_cell(const AdjArgs& a, const LineGeom& g, long long L, int p,
                                          int& i, int& j, int& k) {
  const int n0 = g.d == 0 ? a.ny : a.nx;
  int lo, hi;
  if (g.nlines <= 0xffffffffLL) {
    const unsigned u = (unsigned)L, qq = u / (unsigned)n0;
    hi = (int)qq;
    lo = (int)(u - qq * (unsigned)n0);
  } else {
    hi = (int)(L / n0);
    lo = (int)(L - (long long)hi * n0);
  }
  if (g.d == 0) {
    i = p;
    j = lo;
    k = hi;
  } else if (g.d == 1) {
    i = lo;
    j = p;
    k = hi;
  } else {
    i = lo;
    j = hi;
    k = p;
  }
}

// Optional occupancy target of the fused direction kernel (waves per SIMD);
// 0 leaves the register budget to the compiler.
#ifndef SNAP_ADJ_LINE_WAVES_PER_EU
#define SNAP_ADJ_LINE_WAVES_PER_EU 0
#endif
#if SNAP_ADJ_LINE_WAVES_PER_EU > 0
#define SNAP_ADJ_LINE_ATTR __attribute__((amdgpu_waves_per_eu(SNAP_ADJ_LINE_WAVES_PER_EU)))
#else
#define SNAP_ADJ_LINE_ATTR
#endif

template <typename T, int NV, int LN, int TL, bool XDIR, bool HLLC = false, bool MIX = false>
__global__ void __launch_bounds__((LineTile<T, NV, LN, TL>::NTHR)) SNAP_ADJ_LINE_ATTR
    k_adj_line(const T* __restrict__ q, const T* __restrict__ rb, AdjArgs a, int d,
               T* __restrict__ P) {
  using Tile = LineTile<T, NV, LN, TL>;
  constexpr int NTHR = Tile::NTHR;
  static_assert(NTHR >= LN * Tile::NA, "one item of phase A per thread");
  __shared__ Tile S;
  const LineGeom g = line_geom(a, d);
  const unsigned nseg = (unsigned)((g.nd + TL - 1) / TL);
  const unsigned lt = blockIdx.x / nseg;
  const int seg = (int)(blockIdx.x - lt * nseg);
  const long long L0 = (long long)lt * LN;
  const int c0 = seg * TL;
  const int c1 = min(c0 + TL, g.nd);
  const T eps = static_cast<T>(a.eps), gamma = static_cast<T>(a.gamma);
  // constant indices only: a runtime index into the argument struct would
  // copy it to scratch memory
  const T inv_gm1 = static_cast<T>(a.inv_gm1);
  const T hi = static_cast<T>(d == 0 ? a.dxi[0] : (d == 1 ? a.dxi[1] : a.dxi[2]));
  const bool linear = a.linear != 0;
  // item (l, p) of a phase with np positions: x lines run p fastest, y/z lines l fastest
  auto decode = [&](int it, int np, int& l, int& p) {
    if (XDIR) {
      l = it / np;
      p = it % np;
    } else {
      l = it % LN;
      p = it / LN;
    }
  };
  // line tables: offsets of position 0 of every line of the tile
  if (threadIdx.x < LN && L0 + threadIdx.x < g.nlines) {
    int i, j, k;
    line_cell(a, g, L0 + threadIdx.x, 0, i, j, k);
    S.pbase[threadIdx.x] = padded_off(a, i, j, k);
    S.rbase[threadIdx.x] = (long long)k * a.rz + (long long)j * a.ry + i;
    S.lev[threadIdx.x] = k;
  }
  __syncthreads();
  // (A) this thread's reconstructed cell jg = c0-3+pa (one per thread, -1 .. nd);
  // the forward quantities stay in registers for its reverse in (C)
  int la, pa;
  decode(threadIdx.x, Tile::NA, la, pa);
  const bool line_a = threadIdx.x < LN * Tile::NA && L0 + la < g.nlines;
  const int ja = c0 - 3 + pa;
  const bool cell_a = line_a && ja >= -1 && ja <= g.nd;
  WenoLin<T> lin[NV];
  // the primitives of the tile's lines, cells c0-5 .. c0+TL+4 (those outside
  // the padded range -3 .. nd+2 are never read), converted from the
  // ghost-filled state and staged in LDS once: the stencils of (A) and (C)
  // are read from there
  for (int it = threadIdx.x; it < LN * (TL + 10); it += NTHR) {
    int l, m;
    decode(it, TL + 10, l, m);
    const int jg = c0 - 5 + m;
    if (L0 + l < g.nlines && jg >= -3 && jg <= g.nd + 2) {
      const long long pc = S.pbase[l] + jg * g.sd;
      const int kl = d == 2 ? jg : S.lev[l];   // level of the cell
      T x[NV];
      load_prim<T, NV, MIX>(q, pc, a.sv, level_ref(a.pert, a.rbar_c[kl + NG], a.pbar_c[kl + NG]),
                            a.gm1, a.mix, x);
#pragma unroll
      for (int v = 0; v < NV; ++v) S.WL[v][l][m] = x[v];
    }
  }
  __syncthreads();
  // cell ja = c0-3+pa uses cells ja-2 .. ja+2, positions pa .. pa+4 of WL
  auto load_stencils = [&](T (&st)[NV][5]) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int o = 0; o < 5; ++o) st[v][o] = S.WL[v][la][pa + o];
  };
  if (cell_a) {
    T st[NV][5];
    load_stencils(st);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T qm, qp;
      weno5_lin<T>(st[v][0], st[v][1], st[v][2], st[v][3], st[v][4], eps, linear, lin[v], qm, qp);
      S.QM[v][la][pa] = qm;
      S.QP[v][la][pa] = qp;
    }
  }
  __syncthreads();
  // (B) LMARS forward + reverse at faces f = c0-2 .. c0+TL+2 that exist (0 .. nd)
  for (int it = threadIdx.x; it < LN * Tile::NF; it += NTHR) {
    int l, p;
    decode(it, Tile::NF, l, p);
    const int fg = c0 - 2 + p;
    if (L0 + l >= g.nlines) continue;
    T xlb[NV], xrb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xlb[v] = T(0);
      xrb[v] = T(0);
    }
    if (fg >= 0 && fg <= g.nd) {
      T xl[NV], xr[NV], fbar[NV];
      // face fg: left state = qm of cell fg-1 (index p), right = qp of cell fg (index p+1)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        xl[v] = S.QM[v][l][p];
        xr[v] = S.QP[v][l][p + 1];
      }
      const long long ro = S.rbase[l] + (fg < g.nd ? fg : g.nd - 1) * g.rd;   // cell min(fg, nd-1)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T right = fg < g.nd ? rb[ro + v * a.rv] : T(0);
        const long long lo = fg < g.nd ? ro - g.rd : ro;   // cell fg-1
        const T left = fg > 0 ? rb[lo + v * a.rv] : T(0);
        fbar[v] = (right - left) * hi;
      }
      T rref, pref;
      if (d == 2) {
        rref = static_cast<T>(a.rbar_f[fg]);
        pref = static_cast<T>(a.pbar_f[fg]);
      } else {
        rref = static_cast<T>(a.rbar_c[S.lev[l] + NG]);
        pref = static_cast<T>(a.pbar_c[S.lev[l] + NG]);
      }
      riemann_flux_adj<T, NV, HLLC, MIX>(xl, xr, d + 1, rref, pref, gamma, inv_gm1,
                                         static_cast<T>(a.gm1), a.mix, fbar, xlb, xrb);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      S.XL[v][l][p] = xlb[v];
      S.XR[v][l][p] = xrb[v];
    }
  }
  __syncthreads();
  // (C) WENO5 reverse of the same cell: C index pa-1 covers cells c0-2 .. c0+TL+1
  if (line_a && pa >= 1 && pa <= Tile::NC) {
    const int pc = pa - 1;
    if (cell_a) {
      T st[NV][5];
      load_stencils(st);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // qm_j is the left state of face j+1 (XL index pc+1); qp_j the right state of face j (XR index pc)
        const T gm = S.XL[v][la][pc + 1];
        const T gp = S.XR[v][la][pc];
        T out[5];
        weno5_rev<T>(st[v][0], st[v][1], st[v][2], st[v][3], st[v][4], linear, lin[v], gm, gp,
                     out);
#pragma unroll
        for (int o = 0; o < 5; ++o) S.C[o][v][la][pc] = out[o];
      }
    } else {
#pragma unroll
      for (int o = 0; o < 5; ++o)
#pragma unroll
        for (int v = 0; v < NV; ++v) S.C[o][v][la][pc] = T(0);
    }
  }
  __syncthreads();
  // (D) cells of the tile, plus the ghost cells beyond a domain edge
  const int lo = c0 == 0 ? -3 : c0;
  const int hiend = c1 == g.nd ? g.nd + 3 : c1;
  const int npos = hiend - lo;
  for (int it = threadIdx.x; it < LN * (TL + 6); it += NTHR) {
    int l, p;
    decode(it, TL + 6, l, p);
    if (p >= npos || L0 + l >= g.nlines) continue;
    const int cg = lo + p;
    const long long pc = S.pbase[l] + cg * g.sd;
    // the first direction kernel to reach a cell starts its sum from zero: x
    // reaches every cell of the interior rows (x ghosts included), y and z
    // the ghost cells beyond their own edges first (no zero-fill pass)
    const bool first = XDIR || cg < 0 || cg >= g.nd;
    T acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = first ? T(0) : P[pc + v * a.sv];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int jg = cg + 2 - o;   // reconstruction whose input o is this cell
      if (jg < -1 || jg > g.nd) continue;
      const int q = jg - (c0 - 2);   // its index in C
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += S.C[o][v][l][q];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) P[pc + v * a.sv] = acc[v];
  }
}

__device__ __forceinline__ int adj_ghost_src(int idx, int n, int bc) {
  if (idx >= 0 && idx < n) return idx;
  if (bc == 0) return ((idx % n) + n) % n;
  if (idx < 0) return min(-1 - idx, n - 1);
  return max(2 * n - 1 - idx, 0);
}

// Before a folding z march (single precision, after the x direction): each
// interior cell within 3 of an x edge takes the primitive cotangents of the
// ghost cells that copy it in x into its own (fixed order: low then high
// ghost positions). A periodic copy holds the cell's state and a mirror copy
// the state with the normal momentum negated, i.e. the primitives with the
// normal velocity negated, so by the chain rule the copy's cotangent (its x
// velocity component negated for a mirror) adds to the cell's primitive
// cotangent before the reverse of the conserved -> primitive map; the fold
// then skips the copies in x. P of the ghost cells is final once the x
// direction has run: the y and z directions write no cell outside the
// interior in x. Grid: one thread per edge cell (min(nx, 6) per row), rows
// over the interior.
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_xmerge(T* __restrict__ P, AdjArgs a) {
  const int ne = a.nx > 6 ? 6 : a.nx;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)ne * a.ny * a.nz) return;
  const int e = (int)(t % ne), row = (int)(t / ne);
  const int i = a.nx > 6 && e >= 3 ? a.nx - 6 + e : e;
  const int j = row % a.ny, k = row / a.ny;
  const long long c = padded_off(a, i, j, k);
  T pv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) pv[v] = P[c + v * a.sv];
  const bool flip = a.bc[0] == 1;
  for (int m = 0; m < 6; ++m) {
    const int gidx = m < 3 ? -1 - m : a.nx + (m - 3);
    if (adj_ghost_src(gidx, a.nx, a.bc[0]) != i) continue;
    const long long g = c + (gidx - i);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T x = P[g + v * a.sv];
      pv[v] += (flip && v == 1) ? -x : x;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) P[c + v * a.sv] = pv[v];
}

// Where the z march stores the conserved cotangent of the cells it folds:
// out (interior layout) overwritten (mode 0), added to (mode 1),
// out = alpha * out + beta * result (mode 2), out = alpha * rb + beta * result
// (mode 3), out = alpha * out + gam * y + rb + beta * result (mode 4); out ==
// nullptr: no fold (the march writes P for every cell).
template <typename T>
struct MarchFold {
  T* out;
  const T* y;
  int mode;
  T alpha, beta, gam;
};

// Fold of one interior cell at least 3 cells from the y and z edges (level
// k), in the precision of the march, from its complete primitive cotangent own
// (in registers; for a cell within 3 of an x edge k_adj_xmerge has added the
// cotangents of its copies in x) and its primitives x (the march's window):
// gravity and the reverse of the conserved -> primitive map as adj_cons_cell
// does for the passive gas, and the store by the fold's mode. bo, ro: byte
// offsets of the cell in a padded and in an interior plane.
template <typename T, int NV>
__device__ __forceinline__ void fold_march_cell(const T* __restrict__ q,
                                                const T* __restrict__ rb, const AdjArgs& a,
                                                const MarchFold<T>& fo, const T (&x)[NV],
                                                const T (&own)[NV], unsigned bo, unsigned ro,
                                                int k) {
  auto at = [](const T* base, unsigned boff) -> const T& {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
  };
  T pv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) pv[v] = own[v];
  const T inv = rcp_fast(at(q, bo) + static_cast<T>(a.pert ? a.rbar_c[k + NG] : 0.0));
  const T u = x[1], v = x[2], w = x[3];
  const T grav = static_cast<T>(a.grav);
  pv[0] -= grav * at(rb + 3 * a.rv, ro);          // R_rhow -= g rho'
  const T qe = -grav * at(rb + 4 * a.rv, ro);     // R_E -= g rho w
  const T Qb = static_cast<T>(a.gm1) * pv[4];
  T o[NV];
  T rhob = pv[0] - (u * pv[1] + v * pv[2] + w * pv[3]) * inv + Qb * T(0.5) * (u * u + v * v + w * w);
#pragma unroll
  for (int t = 5; t < NV; ++t) {
    rhob -= x[t] * pv[t] * inv;
    o[t] = pv[t] * inv;
  }
  o[0] = rhob;
  o[1] = pv[1] * inv - Qb * u;
  o[2] = pv[2] * inv - Qb * v;
  o[3] = pv[3] * inv - Qb * w + qe;
  o[4] = Qb;
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    T* op = reinterpret_cast<T*>(reinterpret_cast<char*>(fo.out + m * a.rv) + ro);
    if (fo.mode == 0)
      *op = o[m];
    else if (fo.mode == 1)
      *op = *op + o[m];
    else if (fo.mode == 2)
      *op = fo.alpha * *op + fo.beta * o[m];
    else if (fo.mode == 3)
      *op = fo.alpha * at(rb + m * a.rv, ro) + fo.beta * o[m];
    else
      *op = fo.alpha * *op + fo.gam * at(fo.y + m * a.rv, ro) + at(rb + m * a.rv, ro) +
            fo.beta * o[m];
  }
}

// ---------------------------------------------------------------------------
// Adjoint of one direction D (1 = y, 2 = z) by a march along the lines: one
// thread per segment [c0, c1) of a line, the threads of a wave on consecutive
// x cells (every load and store coalesced), stepping through the cells in
// order with the primitives of six consecutive cells, the cotangent sums of
// five, and the previous cell's left face state, right-state cotangent and
// r_bar in registers: no LDS and no barrier. At cell j the thread
//   (1) reconstructs cell j (weno5_cell: its two face values);
//   (2) evaluates LMARS forward and reverse at face j, between cells j-1 and
//       j, with the flux cotangent (r_bar[j] - r_bar[j-1]) / dx_D;
//   (3) runs the WENO5 reverse of cell j-1 (weno5_linrev, which recomputes
//       that cell's weights) with the cotangents of its face values from
//       faces j and j-1, and adds the five contributions to the sums of
//       cells j-3 .. j+1;
//   (4) writes the sum of cell j-3, now complete, into P.
// Each sum has one fixed order (P as the previous direction left it, or zero
// for a ghost cell beyond this direction's edges, then the contributions of
// reconstructions j-2 .. j+2 in turn), so the result is reproducible bit for
// bit. A segment recomputes the reconstructions and faces of a 3-cell halo on
// each side; the ghost cells beyond a domain edge belong to the first or the
// last segment of the line.
// Grid: x over blocks of 256 lines (x fastest), y over segments of seglen.
// With 5 variables held to three waves per SIMD (168 registers: the y
// instance would otherwise take 169); with 6 or 7 to two, whose window does
// not fit 168 registers without spills.
// ---------------------------------------------------------------------------
template <typename T, int NV, int D, bool HLLC = false>
__global__ void __launch_bounds__(256, NV <= 5 ? 3 : 2) k_adj_march(const T* __restrict__ q,
                                                   const T* __restrict__ rb, AdjArgs a,
                                                   int seglen, T* __restrict__ P,
                                                   MarchFold<T> fo) {
  static_assert(D == 1 || D == 2, "march directions: y and z");
  const int n1 = D == 2 ? a.ny : a.nz;   // second transverse extent
  const int nd = D == 2 ? a.nz : a.ny;   // cells along the line
  const long long line = (long long)blockIdx.x * 256 + threadIdx.x;
  if (line >= (long long)a.nx * n1) return;
  const int i = (int)(line % a.nx), o1 = (int)(line / a.nx);
  const int c0 = (int)blockIdx.y * seglen;
  if (c0 >= nd) return;
  const int c1 = min(c0 + seglen, nd);
  const long long sd = D == 2 ? a.sz : a.sy;
  const long long rd = D == 2 ? a.rz : a.ry;
  // padded offset of position 0 of the line, interior offset of position 0
  const long long pb = D == 2 ? padded_off(a, i, o1, 0) : padded_off(a, i, 0, o1);
  const long long rbo = D == 2 ? (long long)o1 * a.ry + i : (long long)o1 * a.rz + i;
  const T eps = static_cast<T>(a.eps), gamma = static_cast<T>(a.gamma);
  const T inv_gm1 = static_cast<T>(a.inv_gm1);
  const T hi_d = static_cast<T>(D == 2 ? a.dxi[2] : a.dxi[1]);
  const bool linear = a.linear != 0;
  // y faces take the reference of the line's level
  const T rref_c = D == 1 ? static_cast<T>(a.rbar_c[o1 + NG]) : T(0);
  const T pref_c = D == 1 ? static_cast<T>(a.pbar_c[o1 + NG]) : T(0);

  const int jA = max(c0 - 3, -1);                       // first reconstructed cell
  const int jL = min(c1 + 2, nd);                       // last reconstructed cell
  const int fA = max(c0 - 2, 0), fB = min(c1 + 2, nd);  // faces
  const int rA = max(c0 - 2, -1), rB = min(c1 + 1, nd); // reversed reconstructions
  const int lo = c0 == 0 ? -3 : c0, hi = c1 == nd ? nd + 3 : c1;   // cells written
  T win[6][NV];   // primitives of cells j-3 .. j+2
  T acc[5][NV];   // cotangent sums of cells j-3 .. j+1
  T qmp[NV], gpp[NV], rbp[NV];
  // Every access is a uniform per-variable base (q, P: padded planes; r_bar:
  // interior planes) plus one 32-bit byte offset per cell, which the caller
  // keeps below 2^31 (each variable's plane is smaller than 2 GiB).
  auto at = [](const T* base, unsigned boff) -> const T& {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
  };
  const unsigned bsd = (unsigned)(sd * (long long)sizeof(T));
  const unsigned brd = (unsigned)(rd * (long long)sizeof(T));
  // primitives of cell c of the line (padded range -3 .. nd+2), converted
  // from the ghost-filled state with the references of its level
  auto prims = [&](int c, T (&x)[NV]) {
    const int kl = D == 2 ? c : o1;
    const unsigned bo = (unsigned)(pb * (long long)sizeof(T)) + (unsigned)c * bsd;
    T cv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cv[v] = at(q + v * a.sv, bo);
    const LevelRef lr = level_ref(a.pert, a.rbar_c[kl + NG], a.pbar_c[kl + NG]);
    cons_to_prim_sp<NV>(cv, lr.ra, lr.rs, lr.ps, a.gm1, x);
  };
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int cw = jA - 3 + m;
    if (cw >= -3) {
      prims(cw, win[m]);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) win[m][v] = T(0);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    win[5][v] = T(0);
#pragma unroll
    for (int m = 0; m < 5; ++m) acc[m][v] = T(0);   // cells jA-3 .. jA: ghosts or not written
    qmp[v] = T(0);
    gpp[v] = T(0);
    rbp[v] = T(0);
  }
  for (int j = jA; j <= hi + 2; ++j) {
    // loads: primitives of cell j+2, r_bar of cell j, P of cell j+1 (start of its sum)
    if (j <= nd) prims(j + 2, win[5]);
    T rbc[NV];
    const bool rin = j >= 0 && j < nd && j <= fB;
    {
      const unsigned bo = (unsigned)(rbo * (long long)sizeof(T)) + (unsigned)j * brd;
#pragma unroll
      for (int v = 0; v < NV; ++v) rbc[v] = rin ? at(rb + v * a.rv, bo) : T(0);
    }
    {
      const int cn = j + 1;
      const bool from_p = cn >= lo && cn < hi && cn >= 0 && cn < nd;
      const unsigned bo = (unsigned)(pb * (long long)sizeof(T)) + (unsigned)cn * bsd;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[4][v] = from_p ? at(P + v * a.sv, bo) : T(0);
    }
    // (1) face values of cell j
    T qm[NV], qp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qm[v] = T(0);
      qp[v] = T(0);
    }
    if (j <= jL) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        weno5_cell<T>(win[1][v], win[2][v], win[3][v], win[4][v], win[5][v], eps, linear, qm[v],
                      qp[v]);
    }
    // (2) face j: left state qm of cell j-1, right state qp of cell j
    T xlb[NV], xrb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xlb[v] = T(0);
      xrb[v] = T(0);
    }
    if (j >= fA && j <= fB) {
      T fbar[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) fbar[v] = (rbc[v] - rbp[v]) * hi_d;
      const T rref = D == 2 ? static_cast<T>(a.rbar_f[j]) : rref_c;
      const T pref = D == 2 ? static_cast<T>(a.pbar_f[j]) : pref_c;
      riemann_flux_adj<T, NV, HLLC, false>(qmp, qp, D + 1, rref, pref, gamma, inv_gm1,
                                           static_cast<T>(a.gm1), a.mix, fbar, xlb, xrb);
    }
    // (3) reverse of cell j-1 (stencil cells j-3 .. j+1)
    if (j - 1 >= rA && j - 1 <= rB) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T g[5];
        weno5_linrev<T>(win[0][v], win[1][v], win[2][v], win[3][v], win[4][v], eps, linear,
                        xlb[v], gpp[v], g);
#pragma unroll
        for (int o = 0; o < 5; ++o) acc[o][v] += g[o];
      }
    }
    // (4) cell j-3 is complete: folded (z march, cells at least 3 from the
    // y and z edges) or written into P
    {
      const int cf = j - 3;
      if (cf >= lo && cf < hi) {
        const unsigned bo = (unsigned)(pb * (long long)sizeof(T)) + (unsigned)cf * bsd;
        bool folded = false;
        if constexpr (D == 2) {
          if (fo.out != nullptr && cf >= 3 && cf < nd - 3 &&
              (!a.d3 || (o1 >= 3 && o1 < a.ny - 3))) {
            fold_march_cell<T, NV>(q, rb, a, fo, win[0], acc[0], bo,
                                   (unsigned)(rbo * (long long)sizeof(T)) + (unsigned)cf * brd, cf);
            folded = true;
          }
        }
        if (!folded) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
            *reinterpret_cast<T*>(reinterpret_cast<char*>(P + v * a.sv) + bo) = acc[0][v];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int m = 0; m < 5; ++m) win[m][v] = win[m + 1][v];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m][v] = acc[m + 1][v];
      qmp[v] = qm[v];
      gpp[v] = xrb[v];
      rbp[v] = rbc[v];
    }
  }
}

// Conserved cotangent of one cell of the stencil region (interior
// coordinates; ghost cells lie outside the domain along one axis at most),
// in double precision: gravity terms (interior cells only) and the reverse of
// the conserved -> primitive map applied to the primitive cotangent P.
// Passive gas: p = (gamma - 1)(E - K). Mixture (MIX, App. B):
// p = (gamma - 1)(n / d)((E - K) - A) with n = 1 + sum a_t q_t,
// d = 1 + sum b_t q_t, A = sum mu_t rho_t and q_t = rho_t / rho; with
// Qb = (gamma - 1)(n / d) pb_p the cotangents of E, of the momenta through K
// and of the tracer densities through A are Qb, -Qb u_i and -Qb mu_t, and
// n / d adds ((gamma - 1) Q pb_p)(a_t / d - b_t n / d^2) to each fraction's
// cotangent, Q = (E - K) - A. The passive form is the case n = d = 1, A = 0.
template <typename T, int NV, bool MIX>
__device__ __forceinline__ void adj_cons_cell(const T* __restrict__ q, const T* __restrict__ P,
                                              const T* __restrict__ rb, const AdjArgs& a, int i,
                                              int j, int k, double (&out)[NV]) {
  const long long c = padded_off(a, i, j, k);
  double pb[NV], cv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    pb[v] = static_cast<double>(P[c + v * a.sv]);
    cv[v] = static_cast<double>(q[c + v * a.sv]);
  }
  double qe = 0.0;   // extra conserved cotangent of rho w from the energy source
  const bool inside = i >= 0 && i < a.nx && j >= 0 && j < a.ny && k >= 0 && k < a.nz;
  if (inside) {
    const long long ro = (long long)k * a.rz + (long long)j * a.ry + i;
    pb[0] += -a.grav * static_cast<double>(rb[ro + 3 * a.rv]);   // R_rhow -= g rho'
    qe = -a.grav * static_cast<double>(rb[ro + 4 * a.rv]);       // R_E -= g rho w
  }
  // rho of the cell (perturbation storage: the stored value plus rhobar of its level)
  const double inv = 1.0 / (cv[0] + (a.pert ? a.rbar_c[k + NG] : 0.0));
  const double u = cv[1] * inv, v = cv[2] * inv, w = cv[3] * inv;
  double Qb = a.gm1 * pb[4];   // cotangent of (E - K) - A
  double fb[NV];               // extra cotangents of the fractions (mixture)
#pragma unroll
  for (int t = 5; t < NV; ++t) fb[t] = 0.0;
  if constexpr (MIX) {
    constexpr int NT = NV - 5;
    double num = 1.0, den = 1.0, A = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double qt = cv[5 + t] * inv;
      num += a.mix.a[t] * qt;
      den += a.mix.b[t] * qt;
      A += a.mix.mu[t] * cv[5 + t];
    }
    const double K = 0.5 * (cv[1] * u + cv[2] * v + cv[3] * w);
    const double R = num / den, Q = (cv[4] - K) - A;
    const double Rb = a.gm1 * Q * pb[4];
    Qb = a.gm1 * R * pb[4];
#pragma unroll
    for (int t = 0; t < NT; ++t) fb[5 + t] = Rb * (a.mix.a[t] - a.mix.b[t] * R) / den;
  }
  // p from E - K: dp/drho = Qb |u|^2 / 2, dp/dm = -Qb u
  double rhob = pb[0] - (u * pb[1] + v * pb[2] + w * pb[3]) * inv +
                Qb * 0.5 * (u * u + v * v + w * w);
#pragma unroll
  for (int t = 5; t < NV; ++t) {
    const double qt = cv[t] * inv;
    const double tb = pb[t] + fb[t];
    rhob -= qt * tb * inv;
    out[t] = tb * inv;
    if constexpr (MIX) out[t] -= Qb * a.mix.mu[t - 5];
  }
  out[0] = rhob;
  out[1] = pb[1] * inv - Qb * u;
  out[2] = pb[2] * inv - Qb * v;
  out[3] = pb[3] * inv - Qb * w + qe;
  out[4] = Qb;
}

// ---------------------------------------------------------------------------
// Reverse of the sedimentation terms (Sec. 2; sediment_cell in the stage
// kernels): condensate t with vertical velocity w_t carries through every z
// face the mass flux m = w_t rho q_t of the cell it comes from (the cell above
// when it falls, below when it rises; none through a closed boundary into the
// domain), with the momentum m (u, v, w) and the energy m e, e = c_t T + K +
// mu_t, T = p / (R_d rho (1 + sum_s a_s q_s)), K = |u|^2 / 2; and heats the
// air of its cell by -g w_t rho q_t. A face's flux F enters R of the cell
// above it with +F / dz and of the cell below with -F / dz, so its cotangent
// is (r_bar[above] - r_bar[below]) / dz (zero for a cell outside the domain),
// and it depends on the primitives of its source cell only: each cell (the
// levels -1 .. nz, for the ghost cells a flux can come from) gathers the
// faces it is the source of, one per condensate, and adds their reverse, and
// that of its heating, to its primitive cotangent in P (after the direction
// kernels, before the fold; double precision).
// Grid: x over rows of the levels -1 .. nz, y over the interior row.
// ---------------------------------------------------------------------------
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_sediment(const T* __restrict__ q,
                                                      const T* __restrict__ rb, AdjArgs a,
                                                      T* __restrict__ P) {
  constexpr int NT = NV - 5;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  const int j = row % a.ny, u_lev = row / a.ny - 1;   // level -1 .. nz
  const long long c = padded_off(a, i, j, u_lev);
  T xt[NV];
  load_prim<T, NV, true>(q, c, a.sv, level_ref(0, a.rbar_c[u_lev + NG], a.pbar_c[u_lev + NG]),
                         a.gm1, a.mix, xt);
  double x[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = static_cast<double>(xt[v]);
  const double rho = a.rbar_c[u_lev + NG] + x[0], pres = a.pbar_c[u_lev + NG] + x[4];
  double num = 1.0;
#pragma unroll
  for (int s = 0; s < NT; ++s) num += a.mix.a[s] * x[5 + s];
  const double temp = pres / (a.sed.rd * rho * num);
  const double kin = 0.5 * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  const double dzi = a.dxi[2];
  auto rbv = [&](int v, int k) -> double {
    if (k < 0 || k >= a.nz) return 0.0;
    return static_cast<double>(rb[(long long)k * a.rz + (long long)j * a.ry + i + v * a.rv]);
  };
  double pb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) pb[v] = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double wt = a.sed.wt[t];
    if (wt == 0.0) continue;
    const bool fall = wt < 0.0;
    const double qt = x[5 + t];
    // frictional heating of this cell's air: R_E -= g w_t rho q_t
    if (u_lev >= 0 && u_lev < a.nz) {
      const double hb = -a.grav * wt * rbv(4, u_lev);
      pb[0] += hb * qt;
      pb[5 + t] += hb * rho;
    }
    // the face this cell is the source of: its lower face (falling), upper (rising)
    const int f = fall ? u_lev : u_lev + 1;   // between levels f - 1 and f
    if (f < 0 || f > a.nz) continue;
    if (a.sed.closed_z && ((fall && f == a.nz) || (!fall && f == 0))) continue;
    double Fb[6];
    const int comp[6] = {0, 1, 2, 3, 4, 5 + t};
#pragma unroll
    for (int m = 0; m < 6; ++m) Fb[m] = (rbv(comp[m], f) - rbv(comp[m], f - 1)) * dzi;
    const double mflux = wt * rho * qt;
    const double e = a.sed.ct[t] * temp + kin + a.mix.mu[t];
    const double mb = Fb[0] + Fb[5] + Fb[1] * x[1] + Fb[2] * x[2] + Fb[3] * x[3] + Fb[4] * e;
    const double eb = Fb[4] * mflux;
    pb[1] += Fb[1] * mflux + eb * x[1];
    pb[2] += Fb[2] * mflux + eb * x[2];
    pb[3] += Fb[3] * mflux + eb * x[3];
    const double tb = a.sed.ct[t] * eb;
    pb[0] += mb * wt * qt - tb * temp / rho;
    pb[5 + t] += mb * wt * rho;
    pb[4] += tb / (a.sed.rd * rho * num);
    const double numb = -tb * temp / num;
#pragma unroll
    for (int s = 0; s < NT; ++s) pb[5 + s] += numb * a.mix.a[s];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
    P[c + v * a.sv] = static_cast<T>(static_cast<double>(P[c + v * a.sv]) + pb[v]);
}

// Per interior cell: its conserved cotangent plus those of the ghost cells
// that copy it (fixed order: x, y, z; low then high; the reflected normal
// momentum negated), computed in place from q and P, so no padded conserved
// cotangent is written and read back. out: interior layout, overwritten
// (mode 0), added to (mode 1), out = alpha * out + beta * result (mode 2),
// out = alpha * rb + beta * result (mode 3; out and rb distinct), or
// out = alpha * out + gam * y + rb + beta * result (mode 4: the last stage of
// the RK3 adjoint with its three-term combination; out, y, rb distinct).
template <typename T, int NV, bool MIX = false>
__global__ void __launch_bounds__(256) k_adj_consfold(const T* __restrict__ q,
                                                      const T* __restrict__ P,
                                                      const T* __restrict__ rb, AdjArgs a,
                                                      T* __restrict__ out, int mode,
                                                      double alpha, double beta,
                                                      const T* __restrict__ y, double gam,
                                                      int zedge) {
  // grid: x over interior rows, y over the interior row. zedge (nz > 6, the
  // z march having folded the rest, after k_adj_xmerge): only the rows of the
  // 3 lowest and the 3 highest levels, then (3-D) the rows within 3 of a y
  // edge on the levels between
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  int j, k;
  if (!zedge) {
    j = row % a.ny;
    k = row / a.ny;
  } else if (row < 6 * a.ny) {
    const int e = row / a.ny;
    j = row % a.ny;
    k = e < 3 ? e : a.nz - 6 + e;
  } else {
    const int ye = a.ny > 6 ? 6 : a.ny;   // edge rows per level
    const int r = row - 6 * a.ny, e = r % ye;
    k = 3 + r / ye;
    j = a.ny > 6 && e >= 3 ? a.ny - 6 + e : e;
  }
  const long long c = ((long long)k * a.ny + j) * a.nx + i;
  double acc[NV];
  adj_cons_cell<T, NV, MIX>(q, P, rb, a, i, j, k, acc);
  // (after k_adj_xmerge the copies in x are in P already)
  for (int d = zedge ? 1 : 0; d < 3; ++d) {
    if (d == 1 && !a.d3) continue;
    const int nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
    const int me = d == 0 ? i : (d == 1 ? j : k);
    if (me >= 3 && me < nd - 3) continue;   // no ghost cell copies a cell this deep
    for (int m = 0; m < 6; ++m) {
      const int gidx = m < 3 ? -1 - m : nd + (m - 3);
      if (adj_ghost_src(gidx, nd, a.bc[d]) != me) continue;
      int gc[3] = {i, j, k};
      gc[d] = gidx;
      double x[NV];
      adj_cons_cell<T, NV, MIX>(q, P, rb, a, gc[0], gc[1], gc[2], x);
      const bool flip = a.bc[d] == 1;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += (flip && v == 1 + d) ? -x[v] : x[v];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const long long o = c + v * a.rv;
    if (mode == 0)
      out[o] = static_cast<T>(acc[v]);
    else if (mode == 1)
      out[o] = static_cast<T>(static_cast<double>(out[o]) + acc[v]);
    else if (mode == 2)
      out[o] = static_cast<T>(alpha * static_cast<double>(out[o]) + beta * acc[v]);
    else if (mode == 3)
      out[o] = static_cast<T>(alpha * static_cast<double>(rb[o]) + beta * acc[v]);
    else
      out[o] = static_cast<T>(alpha * static_cast<double>(out[o]) + gam * static_cast<double>(y[o]) +
                              static_cast<double>(rb[o]) + beta * acc[v]);
  }
}

}  // namespace snap
