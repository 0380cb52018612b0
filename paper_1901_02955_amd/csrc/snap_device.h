// Device building blocks of the SNAP right-hand side for gfx950.
//
// cons_to_prim : conserved -> primitive variables of one cell (App. B, with the
//                single-gas reduction that makes tracers passive).
// weno5_cell   : both face values of one cell from its five-cell window
//                (Sec. 4.2, eq. weno5, Jiang-Shu nonlinear weights).
// lmars_flux   : LMARS flux at one face (Sec. 4.1, eqs. rp and ru).
//
// Primitive vector layout x[NV]: 0 = rho - rhobar, 1..3 = u, v, w,
// 4 = p - pbar, 5.. = tracer mass fractions rho_i / rho.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snap {

constexpr int NG = 3;

// Source index along one axis of the cell a ghost cell copies, for index `idx`
// in interior coordinates (ghosts outside [0, n)). Periodic (bc 0): idx mod n.
// Reflecting: the mirror image across the wall (clamped to the interior for
// n < 3), and `flip` is set: the momentum normal to that wall changes sign.
// Shared by the ghost fill and the stage kernel that reads ghosts in place.
__device__ __forceinline__ int ghost_src(int idx, int n, int bc, bool& flip) {
  flip = false;
  if (idx >= 0 && idx < n) return idx;
  if (bc == 0) return ((idx % n) + n) % n;
  flip = true;
  if (idx < 0) return min(-1 - idx, n - 1);
  return max(2 * n - 1 - idx, 0);
}

// ---------------------------------------------------------------------------
// Conserved -> primitive (App. B). The arithmetic runs in double whatever the
// storage type, and in one fixed order with no fused multiply-add, because the
// pressure perturbation p - pbar cancels strongly against the kinetic energy
// and the reference pressure:
//   inv = 1/rho; u = (rho u) inv (v, w alike); K = ((rho u) u + (rho v) v)
//   + (rho w) w, times 1/2; p = (gamma - 1)(E - K); p' = p - pbar;
//   rho' = rho - rhobar; q_i = rho_i inv.
// Stored perturbations (c[0] = rho - rhobar_k, c[4] = E - pbar_k / (gamma -
// 1)) take the same code with ra = rhobar_k (rho = c[0] + ra) and rbar =
// pbar = 0; the full state has ra = 0 (and rho = c[0] exactly).
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void cons_to_prim(const double (&c)[NV], double ra, double rbar,
                                             double pbar, double gm1, double (&x)[NV]) {
#pragma clang fp contract(off)
  const double inv = 1.0 / (c[0] + ra);
  const double u = c[1] * inv;
  const double v = c[2] * inv;
  const double w = c[3] * inv;
  const double K = 0.5 * ((c[1] * u + c[2] * v) + c[3] * w);
  const double p = gm1 * (c[4] - K);
  x[0] = c[0] - rbar;
  x[1] = u;
  x[2] = v;
  x[3] = w;
  x[4] = p - pbar;
#pragma unroll
  for (int t = 5; t < NV; ++t) x[t] = c[t] * inv;
}

// ---------------------------------------------------------------------------
// Mixture equation of state (Sec. 2, eqs. energy and eos; App. B, eq. p2 and
// the effective adiabatic index). Per tracer t: a_t = 1/eps_t - 1 for a vapour
// of molar-mass ratio eps_t, -1 for a condensate (mass without partial
// pressure); b_t = sigma_t - 1 with sigma_t its heat capacity over c_v of the
// dry gas; mu_t its chemical potential per unit mass. With q_t = rho_t / rho:
//   p = (gamma_d - 1) (1 + sum a_t q_t) / (1 + sum b_t q_t) (E - K - A),
//   A = sum mu_t rho_t, and gamma - 1 of the parcel is the factor before (E - K - A).
// ---------------------------------------------------------------------------
constexpr int MAX_TRACERS = 8;

struct Mixture {
  double a[MAX_TRACERS], b[MAX_TRACERS], mu[MAX_TRACERS];
  // single-precision copies for the FP32 face arithmetic: used straight from
  // scalar registers, where converted doubles would take vector registers
  float af[MAX_TRACERS], bf[MAX_TRACERS], muf[MAX_TRACERS];
};

template <typename T, int NT>
__device__ __forceinline__ void mixture_coef(const Mixture& m, int t, T& a, T& b, T& mu) {
  // with few tracers the converted coefficients fit in vector registers
  // (and are hoisted out of the level loop); with more, the scalar copies
  if constexpr (sizeof(T) == 4 && NT >= 5) {
    a = m.af[t];
    b = m.bf[t];
    mu = m.muf[t];
  } else {
    a = static_cast<T>(m.a[t]);
    b = static_cast<T>(m.b[t]);
    mu = static_cast<T>(m.mu[t]);
  }
}

// Sedimentation of condensates (Sec. 2, eq. d3, the momentum and total-energy
// equations): per tracer its signed vertical velocity wt relative to the air
// (0: does not fall) and heat capacity ct; rd the dry gas constant; closed_z:
// the z axis has walls (no condensate enters through them).
struct Sediment {
  int on, closed_z;
  double wt[MAX_TRACERS], ct[MAX_TRACERS], rd;
  float wtf[MAX_TRACERS], ctf[MAX_TRACERS], rdf;
};

// cons_to_prim with the mixture equation of state, in the fixed order
//   A = (mu_1 rho_1 + mu_2 rho_2) + ...; num = (1 + a_1 q_1) + ...; den alike;
//   p = ((gamma_d - 1)(num / den)) ((E - K) - A)
// (double precision, no contraction, as cons_to_prim).
template <int NV>
__device__ __forceinline__ void cons_to_prim_mix(const double (&c)[NV], double rbar, double pbar,
                                                 double gm1, const Mixture& m, double (&x)[NV]) {
#pragma clang fp contract(off)
  constexpr int NT = NV - 5;
  static_assert(NT >= 1 && NT <= MAX_TRACERS, "the mixture needs tracers");
  const double inv = 1.0 / c[0];
  const double u = c[1] * inv;
  const double v = c[2] * inv;
  const double w = c[3] * inv;
  const double K = 0.5 * ((c[1] * u + c[2] * v) + c[3] * w);
#pragma unroll
  for (int t = 5; t < NV; ++t) x[t] = c[t] * inv;
  double A = m.mu[0] * c[5];
  double num = 1.0, den = 1.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t > 0) A = A + m.mu[t] * c[5 + t];
    num = num + m.a[t] * x[5 + t];
    den = den + m.b[t] * x[5 + t];
  }
  const double p = (gm1 * (num / den)) * ((c[4] - K) - A);
  x[0] = c[0] - rbar;
  x[1] = u;
  x[2] = v;
  x[3] = w;
  x[4] = p - pbar;
}

// ---------------------------------------------------------------------------
// Reciprocal and square root for the stencil arithmetic.
// Double precision: the hardware estimate (v_rcp_f64 / v_rsq_f64, about 2^-25
// relative) refined by Newton-Raphson steps, e <- 1 - d r, r <- r + r e for
// the reciprocal, and by the coupled Goldschmidt form g = y h, r = h / 2,
// e = 1/2 - g r, g <- g + g e, r <- r + r e for the reciprocal square root.
// Measured over 2^20 arguments spread over 2^-100 .. 2^100: one step leaves
// at most 11 ulp (reciprocal) and 36 ulp (square root), two steps 0 and 1
// ulp. The stage kernels take one step (SNAP_F64_REFINE_STEPS): the face
// values then stay within a few 1e-15 of the correctly rounded evaluation,
// far inside the 1e-12 parity bar, and the dependent chain that every
// reconstruction and face flux waits on is two FMAs shorter. Single
// precision: the hardware estimates (1 ulp).
// Arguments are positive and normal on every call site.
// ---------------------------------------------------------------------------
#ifndef SNAP_F64_REFINE_STEPS
#define SNAP_F64_REFINE_STEPS 1
#endif
__device__ __forceinline__ double rcp_fast(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  if (SNAP_F64_REFINE_STEPS < 2) return r;
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_fast(float d) { return __builtin_amdgcn_rcpf(d); }

__device__ __forceinline__ double sqrt_fast(double y) {
  const double h = __builtin_amdgcn_rsq(y);
  double g = y * h, r = 0.5 * h;
  double e = fma(-g, r, 0.5);
  g = fma(g, e, g);
  r = fma(r, e, r);
  e = fma(-g, r, 0.5);
  return fma(g, e, g);
}
__device__ __forceinline__ float sqrt_fast(float y) { return y * __builtin_amdgcn_rsqf(y); }

// Sound speed sqrt(gp / rho) from gp = gamma p and the density, written as
// gp h with h = 1 / sqrt(gp rho) (which is also 1 / (rho c)), so no
// reciprocal of rho is needed. Double precision refines the hardware
// reciprocal square root of y = gp rho by SNAP_F64_REFINE_STEPS Goldschmidt
// steps, which carry g -> sqrt(y) and k -> 1 / (2 sqrt(y)) together (the last
// step updates k only); h = 2 k.
__device__ __forceinline__ double sound_speed_h(double gp, double rho, double& h) {
  const double y = gp * rho;
  const double h0 = __builtin_amdgcn_rsq(y);
  double g = y * h0, k = 0.5 * h0;
  double e = fma(-g, k, 0.5);
  if (SNAP_F64_REFINE_STEPS < 2) {
    k = fma(k, e, k);
  } else {
    g = fma(g, e, g);
    k = fma(k, e, k);
    e = fma(-g, k, 0.5);
    k = fma(k, e, k);
  }
  h = k + k;
  return gp * h;
}
__device__ __forceinline__ float sound_speed_h(float gp, float rho, float& h) {
  h = __builtin_amdgcn_rsqf(gp * rho);
  return gp * h;
}
template <typename T>
__device__ __forceinline__ T sound_speed(T gp, T rho) {
  T h;
  return sound_speed_h(gp, rho, h);
}

// ---------------------------------------------------------------------------
// Fifth-order WENO of one cell j from v_{j-2}, .., v_{j+2} = a, b, c, d, e.
//
// qm = left state at face j+1/2 (the paper's I_weno(Q_{i-3}..Q_{i+1}) for
//      face i-1/2 with i = j+1);
// qp = right state at face j-1/2 (I_weno of the mirrored stencil).
//
// Both share the three Jiang-Shu smoothness indicators of cell j (integrals
// of the squared first and second derivatives of the candidate quadratics
// over the cell). The candidate values are written as c plus differences so a
// uniform window returns c exactly; the linear weights are (0.1, 0.6, 0.3) for
// qm and mirrored for qp (the values that turn eq. weno5 into the printed
// fifth-order polynomial interpolant). Nonlinear weights:
//   w_k = (d_k / s_k^2) / sum_m (d_m / s_m^2),  s_k = eps + beta_k,
// evaluated as d_k t_k / sum_m d_m t_m with t_k the product of the other two
// s_m^2. The weights depend only on the ratios of the s_k, so the code uses
// 4 s_k = 4 eps + (13/3) u_k^2 + v_k^2 (beta_k = (13/12) u_k^2 + (1/4) v_k^2):
// two fused multiply-adds and a product per indicator, with u_k the second
// difference of stencil k and v_k its one-sided first-derivative term.
// The candidate values minus c are, per stencil, u_k +- 3 v_k times a factor:
//   left:  (0.05/6)(u0 + 3 v0), 0.05 (u1 - 3 v1), 0.025 (u2 - 3 v2);
//   right: 0.025 (u0 - 3 v0),   0.05 (u1 + 3 v1), (0.05/6)(u2 + 3 v2)
// (the right state's stencil 0 carries weight 0.3 and stencil 2 weight 0.1).
// Taking 0.05 out of numerator and denominator leaves the factors 1/6, 1, 1/2
// (left) and 1/2, 1, 1/6 (right) inside the candidates, where each but the
// two with 1/6 is one fused multiply-add of the differences, and the
// denominators 2 t0 + 12 t1 + 6 t2 and 6 t0 + 12 t1 + 2 t2, which share
// 12 t1. The face value is c + (sum_k t_k A_k) / den with one fused
// multiply-add at the end. Double precision shares one reciprocal between
// both faces (s_k^8 is far inside the exponent range for eps >= 1e-30 and
// beta < 1e30). Single precision first scales the s_k by about 2^-E, E the
// exponent of their maximum: the float whose bits are 0x7F000000 minus the
// maximum's bits, which brings the maximum to [1, 1.125] without isolating the
// exponent field; a common factor leaves the weights unchanged up to the
// rounding of the three products, and keeps the products of the s_k in range.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void weno5_cell(T a, T b, T c, T d, T e, T eps, bool linear, T& qm,
                                           T& qp) {
  const T da = a - c, db = b - c, dd = d - c, de = e - c;
  const T u1 = db + dd, v1 = db - dd;
  // candidate values minus c over 0.05: left A_k, right B_k (stencil k)
  const T A0 = fma(T(2.0 / 3.0), da, T(-7.0 / 3.0) * db);   // (u0 + 3 v0) / 6
  const T B0 = fma(T(5), db, -da);                           // (u0 - 3 v0) / 2
  const T A1 = fma(T(-3), v1, u1), B1 = fma(T(3), v1, u1);
  const T A2 = fma(T(5), dd, -de);                           // (u2 - 3 v2) / 2
  const T B2 = fma(T(2.0 / 3.0), de, T(-7.0 / 3.0) * dd);   // (u2 + 3 v2) / 6
  if (linear) {
    qm = fma(T(0.05), (A0 + A1) + A2, c);
    qp = fma(T(0.05), (B2 + B1) + B0, c);
    return;
  }
  const T k13 = T(13) / T(3), eps4 = T(4) * eps;
  const T u0 = fma(T(-2), db, da), v0 = fma(T(-4), db, da);
  const T u2 = fma(T(-2), dd, de), v2 = fma(T(-4), dd, de);
  T s0 = fma(v0, v0, fma(k13 * u0, u0, eps4));
  T s1 = fma(v1, v1, fma(k13 * u1, u1, eps4));
  T s2 = fma(v2, v2, fma(k13 * u2, u2, eps4));
  if constexpr (sizeof(T) == 4) {
    const float mx = fmaxf(fmaxf(s0, s1), s2);
    const float sc = __uint_as_float(0x7F000000u - __float_as_uint(mx));
    s0 *= sc;
    s1 *= sc;
    s2 *= sc;
  }
  const T q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
  const T t0 = q1 * q2, t1 = q0 * q2, t2 = q0 * q1;
  const T g1 = T(12) * t1;
  const T denm = fma(T(2), t0, fma(T(6), t2, g1));
  const T denp = fma(T(6), t0, fma(T(2), t2, g1));
  const T numm = fma(t0, A0, fma(t1, A1, t2 * A2));
  const T nump = fma(t0, B0, fma(t1, B1, t2 * B2));
  if constexpr (sizeof(T) == 8) {
    const T inv = rcp_fast(denm * denp);
    qm = fma(numm, denp * inv, c);
    qp = fma(nump, denm * inv, c);
  } else {
    qm = fma(numm, rcp_fast(denm), c);
    qp = fma(nump, rcp_fast(denp), c);
  }
}

// ---------------------------------------------------------------------------
// LMARS flux at one face (Sec. 4.1, eqs. rp and ru), returned DOUBLED: f is
// twice the face flux (the callers scale the flux differences by half the
// inverse spacing, see flux_scale), which saves the halvings below.
//
// xl, xr   reconstructed primitive face states (layout above) on the left and
//          right side; density and pressure are perturbations.
// nrm      index of the normal velocity in x (1 = x, 2 = y, 3 = z faces).
// rref, pref  reference density and pressure of the face; full values are
//          rho = rref + rho', p = pref + p'.
// Sound speed c = sqrt(gamma p / rho) from full face values; the acoustic
// impedance rho c is the product of the side averages of rho and c, so with
// RC = (rho_L + rho_R)(c_L + c_R) = 4 rho c the doubled interface pressure and
// velocity are (perturbation pressure):
//   2 p* = (p'_L + p'_R) - (RC / 4) (u_R - u_L)
//   2 u* = (u_L + u_R) - 4 (p'_R - p'_L) / RC
// The advected vector (rho, rho u, rho v, rho w, E + p, rho q_i) comes from the
// upwind side (left if u* > 0, else right; at u* == 0 every advective term is
// zero, so the side does not matter), with E + p = p gamma / (gamma - 1) +
// rho |u|^2 / 2; 2 p* is added to the normal momentum flux.
template <typename T, int NV>
__device__ __forceinline__ void lmars_flux(const T (&xl)[NV], const T (&xr)[NV], int nrm, T rref,
                                           T pref, T gamma, T inv_gm1, T (&f)[NV]) {
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  const T unl = xl[nrm], unr = xr[nrm];
  const T cl = sound_speed(gamma * pl, rl);
  const T cr = sound_speed(gamma * pr, rr);
  const T RC = (rl + rr) * (cl + cr);
  const T pstar2 = fma(T(-0.25) * RC, unr - unl, xl[4] + xr[4]);
  const T ustar2 = fma(T(-4) * (xr[4] - xl[4]), rcp_fast(RC), unl + unr);
  const bool left = ustar2 > T(0);
  const T rs = left ? rl : rr;
  const T ps = left ? pl : pr;
  const T us = left ? xl[1] : xr[1];
  const T vs = left ? xl[2] : xr[2];
  const T ws = left ? xl[3] : xr[3];
  const T H = fma(ps, gamma * inv_gm1, T(0.5) * rs * (us * us + vs * vs + ws * ws));   // E + p
  const T mflux2 = ustar2 * rs;
  f[0] = mflux2;
  f[1] = mflux2 * us;
  f[2] = mflux2 * vs;
  f[3] = mflux2 * ws;
  f[4] = ustar2 * H;
#pragma unroll
  for (int t = 5; t < NV; ++t) f[t] = mflux2 * (left ? xl[t] : xr[t]);
  f[nrm] += pstar2;
}

// HLLC flux at one face (the Riemann solver the paper compares LMARS with):
// Davis outer wave speeds S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L,
// u_R + c_R); contact speed S* = (p_R - p_L + d_L u_L - d_R u_R) / (d_L - d_R)
// with d_K = rho_K (S_K - u_K); flux F_L if 0 <= S_L, F_L + S_L (U*_L - U_L) if
// S_L < 0 <= S*, F_R + S_R (U*_R - U_R) if S* < 0 < S_R, F_R if S_R <= 0, where
// U*_K = d_K / (S_K - S*) (1, S* on the normal and the side's tangential
// velocities, E_K/rho_K + (S* - u_K)(S* + p_K / d_K), q_K). Face states and
// references as for lmars_flux; the normal momentum flux carries the
// perturbation pressure (the full flux minus the face reference pressure).
template <typename T, int NV>
__device__ __forceinline__ void hllc_flux(const T (&xl)[NV], const T (&xr)[NV], int nrm, T rref,
                                          T pref, T gamma, T inv_gm1, T (&f)[NV]) {
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  const T unl = nrm == 1 ? xl[1] : (nrm == 2 ? xl[2] : xl[3]);
  const T unr = nrm == 1 ? xr[1] : (nrm == 2 ? xr[2] : xr[3]);
  const T cl = sound_speed(gamma * pl, rl);
  const T cr = sound_speed(gamma * pr, rr);
  const T SL = fmin(unl - cl, unr - cr), SR = fmax(unl + cl, unr + cr);
  const T dl = rl * (SL - unl), dr = rr * (SR - unr);
  const T Ss = (pr - pl + dl * unl - dr * unr) * rcp_fast(dl - dr);
  // the side whose flux (plain or star) is taken, and whether in the star region
  const bool left = SL >= T(0) || Ss >= T(0);
  const bool star = !(SL >= T(0)) && (left || SR > T(0));
  const T rk = left ? rl : rr, pk = left ? pl : pr, ppk = left ? xl[4] : xr[4];
  const T uk = left ? xl[1] : xr[1], vk = left ? xl[2] : xr[2], wk = left ? xl[3] : xr[3];
  const T unk = left ? unl : unr, Sk = left ? SL : SR, dk = left ? dl : dr;
  const T E = pk * inv_gm1 + T(0.5) * rk * (uk * uk + vk * vk + wk * wk);
  const T mass = rk * unk;
  f[0] = mass;
  f[1] = mass * uk + (nrm == 1 ? ppk : T(0));
  f[2] = mass * vk + (nrm == 2 ? ppk : T(0));
  f[3] = mass * wk + (nrm == 3 ? ppk : T(0));
  f[4] = (E + pk) * unk;
#pragma unroll
  for (int t = 5; t < NV; ++t) f[t] = mass * (left ? xl[t] : xr[t]);
  if (star) {
    const T fac = dk * rcp_fast(Sk - Ss);
    const T e_star = fac * (E * rcp_fast(rk) + (Ss - unk) * (Ss + pk * rcp_fast(dk)));
    f[0] += Sk * (fac - rk);
    f[1] += Sk * (fac * (nrm == 1 ? Ss : uk) - rk * uk);
    f[2] += Sk * (fac * (nrm == 2 ? Ss : vk) - rk * vk);
    f[3] += Sk * (fac * (nrm == 3 ? Ss : wk) - rk * wk);
    f[4] += Sk * (e_star - E);
#pragma unroll
    for (int t = 5; t < NV; ++t) {
      const T qk = left ? xl[t] : xr[t];
      f[t] += Sk * (fac - rk) * qk;
    }
  }
}

// LMARS flux with the mixture equation of state: each side's effective
// gamma - 1 = gm1 n / d with n = 1 + sum a_t q_t, d = 1 + sum b_t q_t of its
// face mass fractions, so c^2 = (d + gm1 n) p / (d rho); the advected energy
// is p d / (gm1 n) + rho |u|^2 / 2 + rho sum mu_t q_t of the upwind side.
template <typename T, int NV>
__device__ __forceinline__ void lmars_flux_mix(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                               T rref, T pref, T gm1, const Mixture& m,
                                               T (&f)[NV]) {
  constexpr int NT = NV - 5;
  const T rl = rref + xl[0], rr = rref + xr[0];
  const T pl = pref + xl[4], pr = pref + xr[4];
  // normal velocities by selects: a runtime index would put the face states
  // in scratch memory
  const T unl = nrm == 1 ? xl[1] : (nrm == 2 ? xl[2] : xl[3]);
  const T unr = nrm == 1 ? xr[1] : (nrm == 2 ? xr[2] : xr[3]);
  T nl = T(1), dl = T(1), ml = T(0), nr = T(1), dr = T(1), mr = T(0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T at, bt, mt;
    mixture_coef<T, NT>(m, t, at, bt, mt);
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
  const T pstar = T(0.5) * (xl[4] + xr[4]) - T(0.5) * rc * (unr - unl);
  const T ustar = T(0.5) * (unl + unr) - (xr[4] - xl[4]) * (T(0.5) * rcp_fast(rc));
  const bool left = ustar > T(0);
  const T rs = left ? rl : rr;
  const T ps = left ? pl : pr;
  const T us = left ? xl[1] : xr[1];
  const T vs = left ? xl[2] : xr[2];
  const T ws = left ? xl[3] : xr[3];
  const T ds = left ? dl : dr;
  const T gs = left ? gnl : gnr;
  const T ms = left ? ml : mr;
  const T E = ps * ds * rcp_fast(gs) + rs * (T(0.5) * (us * us + vs * vs + ws * ws) + ms);
  const T mflux = ustar * rs;
  f[0] = mflux;
  f[1] = mflux * us;
  f[2] = mflux * vs;
  f[3] = mflux * ws;
  f[4] = ustar * (E + ps);
#pragma unroll
  for (int t = 5; t < NV; ++t) f[t] = mflux * (left ? xl[t] : xr[t]);
  f[1] += nrm == 1 ? pstar : T(0);
  f[2] += nrm == 2 ? pstar : T(0);
  f[3] += nrm == 3 ? pstar : T(0);
}

template <typename T, int NT>
__device__ __forceinline__ void sediment_coef(const Sediment& sd, int t, T& wt, T& ct) {
  if constexpr (sizeof(T) == 4 && NT >= 5) {
    wt = sd.wtf[t];
    ct = sd.ctf[t];
  } else {
    wt = static_cast<T>(sd.wt[t]);
    ct = static_cast<T>(sd.ct[t]);
  }
}

// Sedimentation through the two z faces of one cell, and the heating of its
// air, subtracted from / added to its right-hand side R. xb, x0, xa: primitive
// vectors (rho', u, v, w, p', q) of the cells below, the cell, and above,
// with their level references (rb, pb), (r0, p0), (ra, pa). A falling
// condensate (wt < 0) crosses the upper face with the values of the cell
// above and the lower face with this cell's; a rising one the reverse. No
// condensate comes in through a wall (wall_below / wall_above).
template <typename T, int NV>
__device__ __forceinline__ void sediment_cell(const T (&xb)[NV], const T (&x0)[NV],
                                              const T (&xa)[NV], T rb, T pb, T r0, T p0, T ra,
                                              T pa, bool wall_below, bool wall_above,
                                              const Mixture& mx, const Sediment& sd, T dzi,
                                              T grav, T (&R)[NV]) {
  constexpr int NT = NV - 5;
  const T rd = sizeof(T) == 4 ? static_cast<T>(sd.rdf) : static_cast<T>(sd.rd);
  // density, temperature p / (R_d rho (1 + sum a_s q_s)) and kinetic energy per mass
  auto cell = [&](const T (&x)[NV], T rref, T pref, T& rho, T& temp, T& kin) {
    rho = rref + x[0];
    T num = T(1);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      T a, b, mu;
      mixture_coef<T, NT>(mx, t, a, b, mu);
      num += a * x[5 + t];
    }
    temp = (pref + x[4]) * rcp_fast(rd * rho * num);
    kin = T(0.5) * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  };
  T rhob, tb, kb, rho0, t0, k0, rhoa, ta, ka;
  cell(xb, rb, pb, rhob, tb, kb);
  cell(x0, r0, p0, rho0, t0, k0);
  cell(xa, ra, pa, rhoa, ta, ka);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T wt, ct;
    sediment_coef<T, NT>(sd, t, wt, ct);
    if (wt == T(0)) continue;
    T a, b, mu;
    mixture_coef<T, NT>(mx, t, a, b, mu);
    const bool fall = wt < T(0);
    const T own = rho0 * x0[5 + t];
    // upper face: from above if falling
    const T m_up = (fall && wall_above) ? T(0) : wt * (fall ? rhoa * xa[5 + t] : own);
    const T u_up = fall ? xa[1] : x0[1], v_up = fall ? xa[2] : x0[2], w_up = fall ? xa[3] : x0[3];
    const T e_up = ct * (fall ? ta : t0) + (fall ? ka : k0) + mu;
    // lower face: from this cell if falling
    const T m_lo = (!fall && wall_below) ? T(0) : wt * (fall ? own : rhob * xb[5 + t]);
    const T u_lo = fall ? x0[1] : xb[1], v_lo = fall ? x0[2] : xb[2], w_lo = fall ? x0[3] : xb[3];
    const T e_lo = ct * (fall ? t0 : tb) + (fall ? k0 : kb) + mu;
    const T dm = (m_up - m_lo) * dzi;
    R[0] -= dm;
    R[5 + t] -= dm;
    R[1] -= (m_up * u_up - m_lo * u_lo) * dzi;
    R[2] -= (m_up * v_up - m_lo * v_lo) * dzi;
    R[3] -= (m_up * w_up - m_lo * w_lo) * dzi;
    R[4] -= (m_up * e_up - m_lo * e_lo) * dzi;
    R[4] -= grav * wt * own;   // frictional heating by the falling condensate
  }
}

// Block index -> logical tile with consecutive logical tiles on one XCD.
// The hardware hands block b to XCD b % 8; this inverts that so that each XCD
// works on a contiguous range of tiles (neighbours share halos in its L2).
__device__ __forceinline__ int xcd_logical_block(int b, int nblk) {
  constexpr int NXCD = 8;
  const int per = nblk / NXCD, rem = nblk % NXCD;
  const int x = b % NXCD, idx = b / NXCD;
  return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

}  // namespace snap
