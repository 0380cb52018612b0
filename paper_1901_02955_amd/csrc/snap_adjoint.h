// Discrete adjoint of the right-hand side: q_bar = J(q)^T r_bar, where J is
// the Jacobian of the interior right-hand side (Sec. 4, eq. forward with the
// LMARS flux of Sec. 4.1, the WENO5 reconstruction of Sec. 4.2 and the
// conserved -> primitive map of App. B) with respect to the interior state,
// ghost cells being functions of the interior through the boundary conditions.
//
// The reverse sweep is split into gather-only kernels (no atomics, so the
// result is reproducible bit for bit):
//   k_adj_prims      primitives of every padded cell (as in the forward pass);
//   k_adj_faces<d>   per face of direction d: recompute both WENO face states,
//                    LMARS forward and reverse with the flux cotangent
//                    F_bar = (r_bar[right cell] - r_bar[left cell]) / dx_d;
//                    store the cotangents of the two face states;
//   k_adj_recon<d>   per reconstructed cell (one beyond each end of every
//                    line): WENO5 reverse seeded by the cotangents of its two
//                    face values; store the cotangents of its 5 inputs;
//   k_adj_gather<d>  per cell of the line (ghosts included): add the
//                    contributions of the (up to) 5 reconstructions that read
//                    it, in a fixed order, into the primitive cotangent;
//   k_adj_cons       per padded cell: gravity terms and the reverse of the
//                    conserved -> primitive map (double precision);
//   k_adj_fold       per interior cell: its own cotangent plus those of the
//                    ghost cells that copy it (sign flipped on the reflected
//                    normal momentum).
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
// Reverse of weno5_cell (same formulation as the forward): given the
// cotangents gm of qm and gp of qp, return the cotangents of a..e.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void weno5_cell_adj(T a, T b, T c, T d, T e, T eps, bool linear, T gm,
                                               T gp, T (&g)[5]) {
  const T da = a - c, db = b - c, dd = d - c, de = e - c;
  const T m0 = T(2) * da - T(7) * db, m1 = T(2) * dd - db, m2 = T(5) * dd - de;
  const T p0 = T(2) * de - T(7) * dd, p1 = T(2) * db - dd, p2 = T(5) * db - da;
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
    const T k13 = T(13) / T(12);
    const T u0 = da - T(2) * db, v0 = da - T(4) * db;
    const T u1 = db + dd, v1 = db - dd;
    const T u2 = de - T(2) * dd, v2 = de - T(4) * dd;
    T s0 = eps + (k13 * u0 * u0 + T(0.25) * v0 * v0);
    T s1 = eps + (k13 * u1 * u1 + T(0.25) * v1 * v1);
    T s2 = eps + (k13 * u2 * u2 + T(0.25) * v2 * v2);
    // common power-of-two scale (exact; the weights do not depend on it)
    T sc = T(1);
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
    const T idm = T(1) / (n0 + n1 + n2), idp = T(1) / (r0 + r1 + r2);
    const T wm0 = n0 * idm, wm1 = n1 * idm, wm2 = n2 * idm;
    const T wp0 = r0 * idp, wp1 = r1 * idp, wp2 = r2 * idp;
    const T Mm = wm0 * m0 + wm1 * m1 + wm2 * m2;   // 6 (qm - c)
    const T Mp = wp0 * p0 + wp1 * p1 + wp2 * p2;
    mb0 = gm * wm0 * sixth;
    mb1 = gm * wm1 * sixth;
    mb2 = gm * wm2 * sixth;
    pb0 = gp * wp0 * sixth;
    pb1 = gp * wp1 * sixth;
    pb2 = gp * wp2 * sixth;
    // cotangents of the unnormalised weights
    const T gmD = gm * sixth * idm, gpD = gp * sixth * idp;
    const T nb0 = gmD * (m0 - Mm), nb1 = gmD * (m1 - Mm), nb2 = gmD * (m2 - Mm);
    const T rb0 = gpD * (p0 - Mp), rb1 = gpD * (p1 - Mp), rb2 = gpD * (p2 - Mp);
    const T tb0 = T(0.1) * nb0 + T(0.3) * rb2;
    const T tb1 = T(0.6) * nb1 + T(0.6) * rb1;
    const T tb2 = T(0.3) * nb2 + T(0.1) * rb0;
    const T qb0 = tb1 * q2 + tb2 * q1;
    const T qb1 = tb0 * q2 + tb2 * q0;
    const T qb2 = tb0 * q1 + tb1 * q0;
    // s_k (unscaled) cotangent = sc * 2 s'_k qb'_k ; beta_k has the same cotangent
    const T bb0 = sc * T(2) * s0 * qb0;
    const T bb1 = sc * T(2) * s1 * qb1;
    const T bb2 = sc * T(2) * s2 * qb2;
    ub0 = T(2) * k13 * u0 * bb0;
    vb0 = T(0.5) * v0 * bb0;
    ub1 = T(2) * k13 * u1 * bb1;
    vb1 = T(0.5) * v1 * bb1;
    ub2 = T(2) * k13 * u2 * bb2;
    vb2 = T(0.5) * v2 * bb2;
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
  const T cl = sqrt(gamma * pl / rl), cr = sqrt(gamma * pr / rr);
  const T ra = T(0.5) * (rl + rr), ca = T(0.5) * (cl + cr);
  const T rc = ra * ca;
  const T hh = T(1) / (T(2) * rc);
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
  // advected-vector cotangents of the upwind side (zero at u* == 0)
  if (ustar != T(0)) {
    const bool left = ustar > T(0);
    const T(&x)[NV] = left ? xl : xr;
    T(&xb)[NV] = left ? xlb : xrb;
    const T r = left ? rl : rr;
    T phb[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) phb[m] = ustar * fb[m];
    const T k = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    T rb = phb[0] + phb[1] * x[1] + phb[2] * x[2] + phb[3] * x[3] + phb[4] * k;
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      rb += phb[t] * x[t];
      xb[t] += phb[t] * r;
    }
    xb[0] += rb;
    xb[1] += phb[1] * r + phb[4] * r * x[1];
    xb[2] += phb[2] * r + phb[4] * r * x[2];
    xb[3] += phb[3] * r + phb[4] * r * x[3];
    xb[4] += phb[4] * (inv_gm1 + T(1));
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
  // c = sqrt(gamma p / rho): dc/dp = c / (2p), dc/drho = -c / (2 rho)
  xlb[4] += clb * cl / (T(2) * pl);
  rlb += -clb * cl / (T(2) * rl);
  xrb[4] += crb * cr / (T(2) * pr);
  rrb += -crb * cr / (T(2) * rr);
  xlb[0] += rlb;
  xrb[0] += rrb;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Primitives of every padded cell (ghost corners included, harmlessly).
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_prims(const T* __restrict__ q, AdjArgs a,
                                                   T* __restrict__ W) {
  const long long n = a.sv;
  const long long nxp = a.nx + 2 * NG, nyp = a.d3 ? a.ny + 2 * NG : 1;
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    const int kp = (int)(c / (nxp * nyp));
    T x[NV];
    load_prim<T, NV>(q, c, a.sv, a.rbar_c[kp], a.pbar_c[kp], a.gm1, x);
#pragma unroll
    for (int v = 0; v < NV; ++v) W[c + v * a.sv] = x[v];
  }
}

// Face pass of direction d: cotangents of the left and right face states.
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_faces(const T* __restrict__ W,
                                                   const T* __restrict__ rb, AdjArgs a, int d,
                                                   T* __restrict__ S) {
  const DirBox fb = dir_box(a, d, 1);
  const long long sd = d == 0 ? 1 : (d == 1 ? a.sy : a.sz);   // padded stride along d
  const long long rd = d == 0 ? 1 : (d == 1 ? a.ry : a.rz);   // interior stride along d
  const int nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
  const T eps = static_cast<T>(a.eps), gamma = static_cast<T>(a.gamma);
  const T inv_gm1 = static_cast<T>(a.inv_gm1), hi = static_cast<T>(a.dxi[d]);
  const bool linear = a.linear != 0;
  for (long long g = blockIdx.x * 256LL + threadIdx.x; g < fb.total;
       g += (long long)gridDim.x * 256) {
    int x, y, z;
    box_coords(fb, g, x, y, z);
    const int f = d == 0 ? x : (d == 1 ? y : z);   // face f: between cells f-1 and f
    // interior coordinates of the cell right of the face
    const long long pc = padded_off(a, x, y, z);   // cell f (padded, may be ghost nd)
    T xl[NV], xr[NV], fbar[NV], xlb[NV], xrb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T* w = W + v * a.sv + pc;
      T qp_unused, qm_unused;
      // left state: qm of cell f-1 (stencil f-3 .. f+1)
      weno5_cell<T>(w[-3 * sd], w[-2 * sd], w[-sd], w[0], w[sd], eps, linear, xl[v], qp_unused);
      // right state: qp of cell f (stencil f-2 .. f+2)
      weno5_cell<T>(w[-2 * sd], w[-sd], w[0], w[sd], w[2 * sd], eps, linear, qm_unused, xr[v]);
      xlb[v] = T(0);
      xrb[v] = T(0);
    }
    // flux cotangent: R_c = -(F_{c+1} - F_c) / dx  =>  F_bar_f = (r_bar_f - r_bar_{f-1}) / dx
    const long long ro = (long long)z * a.rz + (long long)y * a.ry + x;   // valid if f < nd
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T right = f < nd ? rb[ro + v * a.rv] : T(0);
      const T left = f > 0 ? rb[ro - rd + v * a.rv] : T(0);
      fbar[v] = (right - left) * hi;
    }
    T rref, pref;
    if (d == 2) {
      rref = static_cast<T>(a.rbar_f[f]);
      pref = static_cast<T>(a.pbar_f[f]);
    } else {
      rref = static_cast<T>(a.rbar_c[z + NG]);
      pref = static_cast<T>(a.pbar_c[z + NG]);
    }
    lmars_flux_adj<T, NV>(xl, xr, d + 1, rref, pref, gamma, inv_gm1, fbar, xlb, xrb);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      S[(2 * v) * fb.total + g] = xlb[v];
      S[(2 * v + 1) * fb.total + g] = xrb[v];
    }
  }
}

// Reconstruction pass of direction d: cotangents of the 5 stencil inputs of
// every reconstructed cell j = -1 .. nd (box coordinate j + 1).
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_recon(const T* __restrict__ W,
                                                   const T* __restrict__ S, AdjArgs a, int d,
                                                   T* __restrict__ C) {
  const DirBox rbx = dir_box(a, d, 2);
  const DirBox fb = dir_box(a, d, 1);
  const long long sd = d == 0 ? 1 : (d == 1 ? a.sy : a.sz);
  const int nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
  const T eps = static_cast<T>(a.eps);
  const bool linear = a.linear != 0;
  for (long long g = blockIdx.x * 256LL + threadIdx.x; g < rbx.total;
       g += (long long)gridDim.x * 256) {
    int x, y, z;
    box_coords(rbx, g, x, y, z);
    int c[3] = {x, y, z};
    const int j = c[d] - 1;   // reconstructed cell
    c[d] = j;
    const long long pc = padded_off(a, c[0], c[1], c[2]);
    // face j+1 (left state = qm_j) and face j (right state = qp_j)
    int f1[3] = {c[0], c[1], c[2]}, f0[3] = {c[0], c[1], c[2]};
    f1[d] = j + 1;
    f0[d] = j;
    const bool has1 = j + 1 <= nd;
    const bool has0 = j >= 0;
    const long long g1 = has1 ? box_index(fb, f1[0], f1[1], f1[2]) : 0;
    const long long g0 = has0 ? box_index(fb, f0[0], f0[1], f0[2]) : 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T gm = has1 ? S[(2 * v) * fb.total + g1] : T(0);
      const T gp = has0 ? S[(2 * v + 1) * fb.total + g0] : T(0);
      const T* w = W + v * a.sv + pc;
      T out[5];
      weno5_cell_adj<T>(w[-2 * sd], w[-sd], w[0], w[sd], w[2 * sd], eps, linear, gm, gp, out);
#pragma unroll
      for (int o = 0; o < 5; ++o) C[((long long)o * NV + v) * rbx.total + g] = out[o];
    }
  }
}

// Gather of direction d into the primitive cotangent P (padded layout, every
// cell of the cross-shaped stencil region): P[c] (+)= sum_{o} C[o][j = c + 2 - o].
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_gather(const T* __restrict__ C, AdjArgs a, int d,
                                                    int accumulate, T* __restrict__ P) {
  const DirBox rbx = dir_box(a, d, 2);
  const DirBox gb = dir_box(a, d, 6);   // cells -3 .. nd+2 along d
  const int nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
  for (long long g = blockIdx.x * 256LL + threadIdx.x; g < gb.total;
       g += (long long)gridDim.x * 256) {
    int x, y, z;
    box_coords(gb, g, x, y, z);
    int c[3] = {x, y, z};
    const int cd = c[d] - 3;
    c[d] = cd;
    const long long pc = padded_off(a, c[0], c[1], c[2]);
    T acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = accumulate ? P[pc + v * a.sv] : T(0);
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int j = cd + 2 - o;   // reconstruction whose input o is this cell
      if (j < -1 || j > nd) continue;
      int r[3] = {c[0], c[1], c[2]};
      r[d] = j + 1;
      const long long gr = box_index(rbx, r[0], r[1], r[2]);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += C[((long long)o * NV + v) * rbx.total + gr];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) P[pc + v * a.sv] = acc[v];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_zero(T* __restrict__ p, long long n) {
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256)
    p[c] = T(0);
}

// out = ca * x + cb * y + cc * z over n elements (interior cotangent arrays).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_combine(T* __restrict__ out, const T* x, const T* y,
                                                     const T* z, double ca, double cb, double cc,
                                                     long long n) {
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    double r = ca * static_cast<double>(x[c]);
    if (y) r += cb * static_cast<double>(y[c]);
    if (z) r += cc * static_cast<double>(z[c]);
    out[c] = static_cast<T>(r);
  }
}

// Per padded cell of the stencil region: gravity and the reverse of the
// conserved -> primitive map. Writes the conserved cotangent Qb (padded).
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_cons(const T* __restrict__ q,
                                                  const T* __restrict__ P,
                                                  const T* __restrict__ rb, AdjArgs a,
                                                  T* __restrict__ Qb) {
  const long long n = a.sv;
  const long long nxp = a.nx + 2 * NG, nyp = a.d3 ? a.ny + 2 * NG : 1;
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    const int ip = (int)(c % nxp);
    const long long r = c / nxp;
    const int jp = (int)(r % nyp);
    const int kp = (int)(r / nyp);
    const int i = ip - NG, j = jp - a.gy, k = kp - NG;
    const int gi = (i < 0 || i >= a.nx) + (j < 0 || j >= a.ny) + (k < 0 || k >= a.nz);
    if (gi > 1) {   // corner ghosts are never read by the cross-shaped stencil
#pragma unroll
      for (int v = 0; v < NV; ++v) Qb[c + v * a.sv] = T(0);
      continue;
    }
    double pb[NV], cv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      pb[v] = static_cast<double>(P[c + v * a.sv]);
      cv[v] = static_cast<double>(q[c + v * a.sv]);
    }
    double qe = 0.0;   // extra conserved cotangent of rho w from the energy source
    if (gi == 0) {
      const long long ro = (long long)k * a.rz + (long long)j * a.ry + i;
      pb[0] += -a.grav * static_cast<double>(rb[ro + 3 * a.rv]);   // R_rhow -= g rho'
      qe = -a.grav * static_cast<double>(rb[ro + 4 * a.rv]);       // R_E -= g rho w
    }
    const double inv = 1.0 / cv[0];
    const double u = cv[1] * inv, v = cv[2] * inv, w = cv[3] * inv;
    // p = (gamma - 1)(E - (m.m)/(2 rho)):  dp/drho = (gamma-1) |u|^2 / 2, dp/dm = -(gamma-1) u
    double rhob = pb[0] - (u * pb[1] + v * pb[2] + w * pb[3]) * inv +
                  a.gm1 * 0.5 * (u * u + v * v + w * w) * pb[4];
    double out[NV];
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      const double qt = cv[t] * inv;
      rhob -= qt * pb[t] * inv;
      out[t] = pb[t] * inv;
    }
    out[0] = rhob;
    out[1] = pb[1] * inv - a.gm1 * u * pb[4];
    out[2] = pb[2] * inv - a.gm1 * v * pb[4];
    out[3] = pb[3] * inv - a.gm1 * w * pb[4] + qe;
    out[4] = a.gm1 * pb[4];
#pragma unroll
    for (int t = 0; t < NV; ++t) Qb[c + t * a.sv] = static_cast<T>(out[t]);
  }
}

__device__ __forceinline__ int adj_ghost_src(int idx, int n, int bc) {
  if (idx >= 0 && idx < n) return idx;
  if (bc == 0) return ((idx % n) + n) % n;
  if (idx < 0) return min(-1 - idx, n - 1);
  return max(2 * n - 1 - idx, 0);
}

// Per interior cell: own cotangent plus those of the ghost cells that copy it.
// out: interior layout, overwritten (mode 0), added to (mode 1), or scaled
// sum out = alpha * out + beta * result (mode 2).
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_adj_fold(const T* __restrict__ Qb, AdjArgs a,
                                                  T* __restrict__ out, int mode, double alpha,
                                                  double beta) {
  const long long n = (long long)a.nx * a.ny * a.nz;
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    const int i = (int)(c % a.nx);
    const long long r = c / a.nx;
    const int j = (int)(r % a.ny);
    const int k = (int)(r / a.ny);
    double acc[NV];
    const long long pc = padded_off(a, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = static_cast<double>(Qb[pc + v * a.sv]);
    // ghosts along each axis in the same line (fixed order: x, y, z; low then high)
    for (int d = 0; d < 3; ++d) {
      if (d == 1 && !a.d3) continue;
      const int nd = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
      const int me = d == 0 ? i : (d == 1 ? j : k);
      for (int m = 0; m < 6; ++m) {
        const int gidx = m < 3 ? -1 - m : nd + (m - 3);
        if (adj_ghost_src(gidx, nd, a.bc[d]) != me) continue;
        int gc[3] = {i, j, k};
        gc[d] = gidx;
        const long long pg = padded_off(a, gc[0], gc[1], gc[2]);
        const bool flip = a.bc[d] == 1;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double x = static_cast<double>(Qb[pg + v * a.sv]);
          acc[v] += (flip && v == 1 + d) ? -x : x;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long o = c + v * a.rv;
      if (mode == 0)
        out[o] = static_cast<T>(acc[v]);
      else if (mode == 1)
        out[o] = static_cast<T>(static_cast<double>(out[o]) + acc[v]);
      else
        out[o] = static_cast<T>(alpha * static_cast<double>(out[o]) + beta * acc[v]);
    }
  }
}

}  // namespace snap
