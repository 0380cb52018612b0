// Kessler microphysics (Sec. 3) integrated by backward Euler, one thread per
// interior cell, double-precision arithmetic for either storage type.
#include "snap_internal.h"

namespace snap {

namespace {

// Value of tracer `idx` of c (a runtime index into a register array would put
// the array in scratch memory; compare-and-select over constant indices instead).
template <int NV>
__device__ __forceinline__ double tracer(const double (&c)[NV], int idx) {
  double r = 0.0;
#pragma unroll
  for (int t = 0; t < NV - 5; ++t) r = t == idx ? c[5 + t] : r;
  return r;
}

template <int NV>
__device__ __forceinline__ void set_tracer(double (&c)[NV], int idx, double val) {
#pragma unroll
  for (int t = 0; t < NV - 5; ++t) c[5 + t] = t == idx ? val : c[5 + t];
}

// Entry `idx` of a per-tracer parameter table in the kernel arguments, by
// compare-and-select (a runtime index would copy the argument struct to scratch).
__device__ __forceinline__ double tracer_of(const double (&tab)[MAX_TRACERS], int idx) {
  double r = 0.0;
#pragma unroll
  for (int t = 0; t < MAX_TRACERS; ++t) r = t == idx ? tab[t] : r;
  return r;
}

// Backward-Euler step of (q_v, q_c, q_p) by the Newton iteration of Sec. 3 in
// the regime of the starting point (saturated: q_v > q*).
__device__ __forceinline__ void kessler_solve(const KesslerSpec& sp, double qs, double dt,
                                              int max_iter, double tol, double& xv, double& xc,
                                              double& xp) {
  const double x0v = xv, x0c = xc, x0p = xp;
  const bool sat = x0v > qs;
  const double lim = tol * (x0v + x0c + x0p);
  const double idt = 1.0 / dt;
  for (int it = 0; it < max_iter; ++it) {
    // rates (Sec. 3, eqs. qi .. qi2) and the residual of X = X^n + dt Phi(X)
    const double cond = sat ? sp.k1 * (xv - qs) : 0.0;
    const double evap = sat ? 0.0 : sp.k4 * xp * (qs - xv);
    const double conv = sp.k2 * xc + sp.k3 * xc * xp;
    const double r0 = (-cond + evap) - (xv - x0v) / dt;
    const double r1 = (cond - conv) - (xc - x0c) / dt;
    const double r2 = (-evap + conv) - (xp - x0p) / dt;
    // M = I/dt - dPhi/dX (row 0, column 1 is zero in both regimes)
    const double A = sp.k2 + sp.k3 * xp, B = sp.k3 * xc, ev = sp.k4 * (qs - xv);
    const double m00 = idt - (sat ? -sp.k1 : -sp.k4 * xp);
    const double m02 = -(sat ? 0.0 : ev);
    const double m10 = -(sat ? sp.k1 : 0.0), m11 = idt + A, m12 = B;
    const double m20 = -(sat ? 0.0 : sp.k4 * xp), m21 = -A, m22 = idt - (sat ? B : B - ev);
    // Cramer's rule
    const double c00 = m11 * m22 - m12 * m21;
    const double c10 = m10 * m22 - m12 * m20;
    const double c20 = m10 * m21 - m11 * m20;
    const double det = m00 * c00 + m02 * c20;
    const double idet = 1.0 / det;
    const double d0 = (r0 * c00 + m02 * (r1 * m21 - m11 * r2)) * idet;
    const double d1 = (m00 * (r1 * m22 - m12 * r2) - r0 * c10 + m02 * (m10 * r2 - r1 * m20)) * idet;
    const double d2 = (m00 * (m11 * r2 - r1 * m21) + r0 * c20) * idet;
    xv += d0;
    xc += d1;
    xp += d2;
    if (fmax(fabs(d0), fmax(fabs(d1), fabs(d2))) <= lim) break;
  }
}

}  // namespace

// grid: x over interior rows (nz ny), y over the interior row
template <typename T, int NT>
__global__ void __launch_bounds__(256) k_kessler(T* __restrict__ q, KesslerArgs a) {
  constexpr int NV = 5 + NT;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  const int j = row % a.ny, k = row / a.ny;
  const long long o = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
  double c[NV], x[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = static_cast<double>(q[o + v * a.sv]);
  cons_to_prim_mix<NV>(c, 0.0, 0.0, a.gm1, a.m, x);   // x[4] = p
  double temp;
  {
    // T = p / (R_d (rho_d + sum over vapours rho_i / eps_i)), rho_d = rho - sum rho_t
#pragma clang fp contract(off)
    double st = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) st = st + c[5 + t];
    double gas = c[0] - st;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (a.vap[t]) gas = gas + c[5 + t] / a.eps[t];
    temp = x[4] / (a.rd * gas);
  }
  const double rho = c[0];
#pragma unroll
  for (int s = 0; s < MAX_TRACERS / 3; ++s) {
    if (s >= a.nspecies) break;
    const KesslerSpec& sp = a.s[s];
    // saturation mixing ratio over the cloud (App. D): p* eps / (R_d T) / rho
    const double tt = temp / sp.t_ref;
    const double pstar = sp.p_ref * exp(sp.beta * (1.0 - 1.0 / tt) - sp.delta * log(tt));
    const double qs = pstar * sp.eps / (a.rd * temp) / rho;
    double xv = tracer(c, sp.v) / rho, xc = tracer(c, sp.c) / rho, xp = tracer(c, sp.p) / rho;
    kessler_solve(sp, qs, a.dt, a.max_iter, a.tol, xv, xc, xp);
    set_tracer(c, sp.v, rho * xv);
    set_tracer(c, sp.c, rho * xc);
    set_tracer(c, sp.p, rho * xp);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) q[o + (5 + t) * a.sv] = static_cast<T>(c[5 + t]);
}

// ---------------------------------------------------------------------------
// Adjoint of the Kessler step: the cotangent of the state before the step
// from that of the state after it, per interior cell (the transpose of the
// step's Jacobian, the regime of X^n and the q*, T of the step's start held
// as in the forward step).
// The step's solution X* of G(X*) = Phi(X*; q*) - (X* - X^n) / dt = 0 moves
// by dX* = M^-1 (dX^n / dt + dPhi/dq* dq*), M = I/dt - dPhi/dX at X* (the
// implicit-function derivative: the forward's Newton matrix at its solution).
// Hence with w = M^-T Xb*: Xb^n = w / dt and qb* = (dPhi/dq*) . w, where
// dPhi/dq* = (k1, -k1, 0) when saturated (condensation k1 (q_v - q*)) and
// (k4 q_p, 0, -k4 q_p) when not (evaporation k4 q_p (q* - q_v)).
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void kessler_solve_adj(const KesslerSpec& sp, double qs, double dt,
                                                  bool sat, double xv, double xc, double xp,
                                                  const double (&xb)[3], double (&x0b)[3],
                                                  double& qsb) {
  const double idt = 1.0 / dt;
  const double A = sp.k2 + sp.k3 * xp, B = sp.k3 * xc, ev = sp.k4 * (qs - xv);
  // M (the forward's Newton matrix), m01 = 0
  const double m00 = idt - (sat ? -sp.k1 : -sp.k4 * xp);
  const double m02 = -(sat ? 0.0 : ev);
  const double m10 = -(sat ? sp.k1 : 0.0), m11 = idt + A, m12 = B;
  const double m20 = -(sat ? 0.0 : sp.k4 * xp), m21 = -A, m22 = idt - (sat ? B : B - ev);
  // N = M^T, solved by Cramer's rule
  const double n00 = m00, n01 = m10, n02 = m20;
  const double n10 = 0.0, n11 = m11, n12 = m21;
  const double n20 = m02, n21 = m12, n22 = m22;
  const double c00 = n11 * n22 - n12 * n21;
  const double c01 = n10 * n22 - n12 * n20;
  const double c02 = n10 * n21 - n11 * n20;
  const double idet = 1.0 / (n00 * c00 - n01 * c01 + n02 * c02);
  const double w0 = (xb[0] * c00 - n01 * (xb[1] * n22 - n12 * xb[2]) +
                     n02 * (xb[1] * n21 - n11 * xb[2])) * idet;
  const double w1 = (n00 * (xb[1] * n22 - n12 * xb[2]) - xb[0] * c01 +
                     n02 * (n10 * xb[2] - xb[1] * n20)) * idet;
  const double w2 = (n00 * (n11 * xb[2] - xb[1] * n21) - n01 * (n10 * xb[2] - xb[1] * n20) +
                     xb[0] * c02) * idet;
  x0b[0] = w0 * idt;
  x0b[1] = w1 * idt;
  x0b[2] = w2 * idt;
  qsb = sat ? sp.k1 * (w0 - w1) : sp.k4 * xp * (w0 - w2);
}

}  // namespace

// q: padded state at the start of the step (read only). qb: interior layout,
// in: cotangent of the state after the step, out: that of the state before.
// grid: x over interior rows (nz ny), y over the interior row
template <typename T, int NT>
__global__ void __launch_bounds__(256) k_kessler_adj(const T* __restrict__ q, T* __restrict__ qb,
                                                     KesslerArgs a) {
  constexpr int NV = 5 + NT;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  const int j = row % a.ny, k = row / a.ny;
  const long long o = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
  const long long rv = (long long)a.nx * a.ny * a.nz;
  const long long ro = (long long)row * a.nx + i;
  double c[NV], x[NV], cb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    c[v] = static_cast<double>(q[o + v * a.sv]);
    cb[v] = static_cast<double>(qb[ro + v * rv]);
  }
  // the forward's temperature (as in k_kessler)
  cons_to_prim_mix<NV>(c, 0.0, 0.0, a.gm1, a.m, x);
  double gas, temp;
  {
#pragma clang fp contract(off)
    double st = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) st = st + c[5 + t];
    gas = c[0] - st;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (a.vap[t]) gas = gas + c[5 + t] / a.eps[t];
    temp = x[4] / (a.rd * gas);
  }
  const double rho = c[0], irho = 1.0 / rho;
  // the species' tracers leave the step through X* only: their cotangents
  // restart from zero and gather the X^n path below
  double yb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) yb[v] = cb[v];
#pragma unroll
  for (int s = 0; s < MAX_TRACERS / 3; ++s) {
    if (s >= a.nspecies) break;
    const KesslerSpec& sp = a.s[s];
    set_tracer(cb, sp.v, 0.0);
    set_tracer(cb, sp.c, 0.0);
    set_tracer(cb, sp.p, 0.0);
  }
  double rhob = 0.0, tb = 0.0;
#pragma unroll
  for (int s = 0; s < MAX_TRACERS / 3; ++s) {
    if (s >= a.nspecies) break;
    const KesslerSpec& sp = a.s[s];
    const double tt = temp / sp.t_ref;
    const double pstar = sp.p_ref * exp(sp.beta * (1.0 - 1.0 / tt) - sp.delta * log(tt));
    const double qs = pstar * sp.eps / (a.rd * temp) / rho;
    const double x0[3] = {tracer(c, sp.v) * irho, tracer(c, sp.c) * irho, tracer(c, sp.p) * irho};
    double xv = x0[0], xc = x0[1], xp = x0[2];
    kessler_solve(sp, qs, a.dt, a.max_iter, a.tol, xv, xc, xp);
    // outputs rho X*: cotangents of X* and of rho
    const double ybs[3] = {tracer(yb, sp.v), tracer(yb, sp.c), tracer(yb, sp.p)};
    const double xb[3] = {rho * ybs[0], rho * ybs[1], rho * ybs[2]};
    rhob += xv * ybs[0] + xc * ybs[1] + xp * ybs[2];
    double x0b[3], qsb;
    kessler_solve_adj(sp, qs, a.dt, x0[0] > qs, xv, xc, xp, xb, x0b, qsb);
    // X^n = rho_t / rho
    set_tracer(cb, sp.v, tracer(cb, sp.v) + x0b[0] * irho);
    set_tracer(cb, sp.c, tracer(cb, sp.c) + x0b[1] * irho);
    set_tracer(cb, sp.p, tracer(cb, sp.p) + x0b[2] * irho);
    rhob -= (x0b[0] * x0[0] + x0b[1] * x0[1] + x0b[2] * x0[2]) * irho;
    // q* = p*(T) eps / (R_d T rho): d ln q* / dT = beta t_ref / T^2 - (delta + 1) / T
    tb += qsb * qs * ((sp.beta * sp.t_ref / temp - sp.delta - 1.0) / temp);
    rhob -= qsb * qs * irho;
  }
  // T = p / (R_d gas), gas = rho - sum_t rho_t + sum_vapours rho_t / eps_t
  const double pb = tb / (a.rd * gas);
  const double gasb = -tb * temp / gas;
  rhob += gasb;
#pragma unroll
  for (int t = 0; t < NT; ++t) cb[5 + t] += gasb * ((a.vap[t] ? 1.0 / a.eps[t] : 0.0) - 1.0);
  // p = (gamma - 1) R Q of the mixture (App. B): R = n / d with
  // n = 1 + sum a_t q_t, d = 1 + sum b_t q_t, q_t = rho_t / rho, and
  // Q = (E - K) - sum mu_t rho_t, K = |m|^2 / (2 rho)
  {
    const double u = x[1], v = x[2], w = x[3];
    double num = 1.0, den = 1.0, A = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      num += a.m.a[t] * x[5 + t];
      den += a.m.b[t] * x[5 + t];
      A += a.m.mu[t] * c[5 + t];
    }
    const double K = 0.5 * (c[1] * u + c[2] * v + c[3] * w);
    const double R = num / den, Q = (c[4] - K) - A;
    const double Qb = a.gm1 * R * pb, Rb = a.gm1 * Q * pb;
    cb[1] -= Qb * u;
    cb[2] -= Qb * v;
    cb[3] -= Qb * w;
    cb[4] += Qb;
    rhob += Qb * 0.5 * (u * u + v * v + w * w);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double fb = Rb * (a.m.a[t] - a.m.b[t] * R) / den;   // cotangent of q_t
      cb[5 + t] += fb * irho - Qb * a.m.mu[t];
      rhob -= fb * x[5 + t] * irho;
    }
  }
  cb[0] += rhob;
#pragma unroll
  for (int v = 0; v < NV; ++v) qb[ro + v * rv] = static_cast<T>(cb[v]);
}

// Saturation adjustment (App. D): each vapour / cloud pair brought to phase
// equilibrium at constant volume and energy, one thread per interior cell,
// double-precision arithmetic. The energy available as heat, E - K - sum mu
// rho, and the heat capacity c_vd (rho_d + sum sigma rho) are carried as
// running sums and updated with every transfer; T is their ratio.
// satadj_iterate adjusts the conserved values c of one cell in place, given
// heat0 = E - K, and leaves chem = sum mu rho and cap = c_vd (rho_d + sum sigma
// rho) of the adjusted composition.
template <int NT>
__device__ __forceinline__ void satadj_iterate(double (&c)[5 + NT], const SatAdjArgs& a,
                                               double heat0, double& chem, double& cap) {
  for (int it = 0; it < a.max_iter; ++it) {
    double moved = 0.0;
#pragma unroll
    for (int s = 0; s < MAX_TRACERS / 2; ++s) {
      if (s >= a.nspecies) break;
      const SatAdjSpec& sp = a.s[s];
      double rv = tracer(c, sp.v), rc = tracer(c, sp.c);
      const double tot = rv + rc;
      if (!(tot > 0.0)) continue;
      const double temp = (heat0 - chem) / cap;
      const double tt = temp / sp.t_ref;
      const double lam = sp.beta / tt - sp.delta;          // d ln p* / d ln T
      const double pstar = sp.p_ref * exp(sp.beta * (1.0 - 1.0 / tt) - sp.delta * log(tt));
      const double f = rv * sp.rv * temp - pstar;          // > 0: supersaturated
      if (rc <= 0.0 && f <= 0.0) continue;                  // no cloud and below saturation
      // latent heating per unit mass condensed: dT/dx = -(dmu + T dcap) / cap
      const double dmu = tracer_of(a.mu, sp.c) - tracer_of(a.mu, sp.v);
      const double dcap = a.cvd * (tracer_of(a.sigma, sp.c) - tracer_of(a.sigma, sp.v));
      const double dTdx = -(dmu + temp * dcap) / cap;
      double fp = -sp.rv * temp + rv * sp.rv * dTdx - pstar * lam / temp * dTdx;
      if (!(fp < 0.0)) fp = -sp.rv * temp;                 // keep the step downhill
      double x = -f / fp;
      x = fmin(fmax(x, -rc), rv);
      rv -= x;
      rc += x;
      chem += x * dmu;
      cap += x * dcap;
      set_tracer(c, sp.v, rv);
      set_tracer(c, sp.c, rc);
      moved = fmax(moved, fabs(x) / tot);
    }
    if (moved <= a.tol) break;
  }
}

// E - K and the initial chem and cap of one cell's conserved values.
template <int NT>
__device__ __forceinline__ double satadj_heat(const double (&c)[5 + NT], const SatAdjArgs& a,
                                              double& chem, double& cap) {
  chem = 0.0;
  cap = c[0];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    chem += a.mu[t] * c[5 + t];
    cap += (a.sigma[t] - 1.0) * c[5 + t];
  }
  cap *= a.cvd;
  return c[4] - 0.5 * (c[1] * c[1] + c[2] * c[2] + c[3] * c[3]) / c[0];
}

// grid: x over interior rows (nz ny), y over the interior row
template <typename T, int NT>
__global__ void __launch_bounds__(256) k_satadj(T* __restrict__ q, SatAdjArgs a) {
  constexpr int NV = 5 + NT;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  const int j = row % a.ny, k = row / a.ny;
  const long long o = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
  double c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = static_cast<double>(q[o + v * a.sv]);
  double chem, cap;
  const double heat0 = satadj_heat<NT>(c, a, chem, cap);
  satadj_iterate<NT>(c, a, heat0, chem, cap);
#pragma unroll
  for (int t = 0; t < NT; ++t) q[o + (5 + t) * a.sv] = static_cast<T>(c[5 + t]);
}

// Adjoint of the saturation adjustment: qb <- J^T qb for the cells' conserved
// values (qb in the interior layout), J the derivative of the adjusted state
// with respect to the state before it, by the implicit-function theorem at the
// equilibrium that k_satadj reaches (recomputed here).
// Per pair s the transfer X_s (mass moved from vapour to cloud) either keeps
// cloud, and then solves G_s = (rho_v0 - X_s) R_v T - p*(T) = 0 with T =
// (E - K - sum mu rho - sum_j X_j dmu_j) / (cap0 + sum_j X_j dcap_j), or sits
// on its bound X_s = -rho_c0 (the cloud evaporated). Over the pairs A with
// cloud left, dG/dX = -diag(a) + g t^T with a_s = R_v T, g_s = dG_s/dT and t_j =
// dT/dX_j, a diagonal plus a rank-one term, so the transposed system has the
// closed form
//   gamma = (sum_A g_s Xb_s / a_s) / (1 - sum_A g_s t_s / a_s),
//   lambda_s a_s = t_s gamma + Xb_s,
// Xb_s = qb[cloud] - qb[vapour] the transfer's cotangent. gamma is the
// cotangent of T (held at fixed X), lambda_s a_s that of rho_v0 through G_s,
// and a bound pair's transfer cotangent Xb_s + gamma t_s goes to -rho_c0.
template <typename T, int NT>
__global__ void __launch_bounds__(256) k_satadj_adj(const T* __restrict__ q, T* __restrict__ qb,
                                                    SatAdjArgs a) {
  constexpr int NV = 5 + NT;
  constexpr int NS = MAX_TRACERS / 2;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int row = blockIdx.x;
  const int j = row % a.ny, k = row / a.ny;
  const long long o = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
  const long long rv = (long long)a.nx * a.ny * a.nz;
  const long long ro = (long long)row * a.nx + i;
  double c[NV], cf[NV], cb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    c[v] = static_cast<double>(q[o + v * a.sv]);
    cf[v] = c[v];
    cb[v] = static_cast<double>(qb[ro + v * rv]);
  }
  double chem, cap;
  const double heat0 = satadj_heat<NT>(c, a, chem, cap);
  satadj_iterate<NT>(cf, a, heat0, chem, cap);
  const double temp = (heat0 - chem) / cap;
  double xb[NS], ts[NS];
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s >= a.nspecies) break;
    const SatAdjSpec& sp = a.s[s];
    xb[s] = tracer(cb, sp.c) - tracer(cb, sp.v);
    const double dmu = tracer_of(a.mu, sp.c) - tracer_of(a.mu, sp.v);
    const double dcap = a.cvd * (tracer_of(a.sigma, sp.c) - tracer_of(a.sigma, sp.v));
    ts[s] = -(dmu + temp * dcap) / cap;
    if (tracer(cf, sp.c) > 0.0) {
      const double tt = temp / sp.t_ref;
      const double lam = sp.beta / tt - sp.delta;
      const double pstar = sp.p_ref * exp(sp.beta * (1.0 - 1.0 / tt) - sp.delta * log(tt));
      const double as = sp.rv * temp;
      const double gs = tracer(cf, sp.v) * sp.rv - pstar * lam / temp;
      num += gs * xb[s] / as;
      den += gs * ts[s] / as;
    }
  }
  const double gam = num / (1.0 - den);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s >= a.nspecies) break;
    const SatAdjSpec& sp = a.s[s];
    if (tracer(cf, sp.c) > 0.0)
      set_tracer(cb, sp.v, tracer(cb, sp.v) + ts[s] * gam + xb[s]);
    else
      set_tracer(cb, sp.c, tracer(cb, sp.c) - (xb[s] + gam * ts[s]));
  }
  // T at fixed transfers: numerator E - K - sum mu rho, denominator cap
  const double nb = gam / cap, db = -gam * temp / cap;
  const double irho = 1.0 / c[0];
  const double u = c[1] * irho, v = c[2] * irho, w = c[3] * irho;
  cb[4] += nb;
  cb[1] -= nb * u;
  cb[2] -= nb * v;
  cb[3] -= nb * w;
  cb[0] += nb * 0.5 * (u * u + v * v + w * w) + db * a.cvd;
#pragma unroll
  for (int t = 0; t < NT; ++t) cb[5 + t] += db * a.cvd * (a.sigma[t] - 1.0) - nb * a.mu[t];
#pragma unroll
  for (int m = 0; m < NV; ++m) qb[ro + m * rv] = static_cast<T>(cb[m]);
}

// Sedimentation part of the right-hand side (from the stage input Qs, ghosts
// filled), added to the stage output: R_sed itself in right-hand-side mode,
// cb dt R_sed after the stage combination (which is linear in R). One thread
// walks a chunk of SED_CHUNK levels of one column with the primitives of the
// levels below, at and above the cell in registers, so that every level is
// converted once. grid: x over (row j, chunk), y over blocks of the row.
constexpr int SED_CHUNK = 16;

template <typename T, int NT>
__global__ void __launch_bounds__(256) k_sediment(StageArgs a, int nchunk) {
  constexpr int NV = 5 + NT;
  const double fd = a.cb * stage_dt(a);
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.nx) return;
  const int j = blockIdx.x / nchunk, kc = blockIdx.x % nchunk;
  const int k0 = kc * SED_CHUNK, k1 = min(k0 + SED_CHUNK, a.nz);
  const T* __restrict__ qs = static_cast<const T*>(a.qs);
  const long long col = (long long)(j + a.gy) * a.sy + (i + NG);
  auto prim = [&](int k, T (&x)[NV]) {   // primitives of level k (ghost levels allowed)
    double c[NV], xd[NV];
    const long long o = col + (long long)(k + NG) * a.sz;
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = static_cast<double>(qs[o + v * a.sv]);
    cons_to_prim_mix<NV>(c, a.rbar_c[k + NG], a.pbar_c[k + NG], a.gm1, a.mix, xd);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = static_cast<T>(xd[v]);
  };
  auto ref = [&](const double* r, int k) { return static_cast<T>(r[k + NG]); };
  // only the five dynamic fields and the falling tracers change (a uniform test)
  auto moves = [&](int v) { return v < 5 || a.sed.wt[v - 5] != 0.0; };
  T xb[NV], x0[NV], xa[NV];
  prim(k0 - 1, xb);
  prim(k0, x0);
  T* __restrict__ out = static_cast<T*>(a.out);
  const T f = static_cast<T>(fd);
  for (int k = k0; k < k1; ++k) {
    prim(k + 1, xa);
    T R[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] = T(0);
    const bool wall_lo = a.sed.closed_z && k == 0, wall_up = a.sed.closed_z && k == a.nz - 1;
    sediment_cell<T, NV>(xb, x0, xa, ref(a.rbar_c, k - 1), ref(a.pbar_c, k - 1), ref(a.rbar_c, k),
                         ref(a.pbar_c, k), ref(a.rbar_c, k + 1), ref(a.pbar_c, k + 1), wall_lo,
                         wall_up, a.mix, a.sed, static_cast<T>(a.dzi), static_cast<T>(a.grav), R);
    if (a.rhs_mode) {
      const long long ro = (long long)k * a.rz + (long long)j * a.ry + i;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (moves(v)) out[ro + v * a.rv] += R[v];
    } else {
      const long long po = col + (long long)(k + NG) * a.sz;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (moves(v)) out[po + v * a.sv] += f * R[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xb[v] = x0[v];
      x0[v] = xa[v];
    }
  }
}

template <typename T>
int launch_sediment_t(int ntracer, const StageArgs& a, hipStream_t st) {
  const int nchunk = (a.nz + SED_CHUNK - 1) / SED_CHUNK;
  const dim3 grid((unsigned)(a.ny * nchunk), (unsigned)((a.nx + 255) / 256));
  switch (ntracer) {
#define SNAP_SEDIMENT_CASE(N)                                                       \
  case N:                                                                           \
    hipLaunchKernelGGL((k_sediment<T, N>), grid, dim3(256), 0, st, a, nchunk);      \
    break;
    SNAP_SEDIMENT_CASE(1)
    SNAP_SEDIMENT_CASE(2)
    SNAP_SEDIMENT_CASE(3)
    SNAP_SEDIMENT_CASE(4)
    SNAP_SEDIMENT_CASE(5)
    SNAP_SEDIMENT_CASE(6)
    SNAP_SEDIMENT_CASE(7)
    SNAP_SEDIMENT_CASE(8)
#undef SNAP_SEDIMENT_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sediment(int dtype, int ntracer, const StageArgs& a, hipStream_t st) {
  return dtype == 0 ? launch_sediment_t<double>(ntracer, a, st)
                    : launch_sediment_t<float>(ntracer, a, st);
}

template <typename T>
int launch_kessler_t(int ntracer, T* q, const KesslerArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.ny * a.nz), (unsigned)((a.nx + 255) / 256));
  switch (ntracer) {
#define SNAP_KESSLER_CASE(N)                                                        \
  case N:                                                                           \
    hipLaunchKernelGGL((k_kessler<T, N>), grid, dim3(256), 0, st, q, a);            \
    break;
    SNAP_KESSLER_CASE(3)
    SNAP_KESSLER_CASE(4)
    SNAP_KESSLER_CASE(5)
    SNAP_KESSLER_CASE(6)
    SNAP_KESSLER_CASE(7)
    SNAP_KESSLER_CASE(8)
#undef SNAP_KESSLER_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_kessler(int dtype, int ntracer, void* q, const KesslerArgs& a, hipStream_t st) {
  return dtype == 0 ? launch_kessler_t<double>(ntracer, static_cast<double*>(q), a, st)
                    : launch_kessler_t<float>(ntracer, static_cast<float*>(q), a, st);
}

template <typename T>
int launch_kessler_adj_t(int ntracer, const T* q, T* qb, const KesslerArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.ny * a.nz), (unsigned)((a.nx + 255) / 256));
  switch (ntracer) {
#define SNAP_KESSLER_ADJ_CASE(N)                                                    \
  case N:                                                                           \
    hipLaunchKernelGGL((k_kessler_adj<T, N>), grid, dim3(256), 0, st, q, qb, a);    \
    break;
    SNAP_KESSLER_ADJ_CASE(3)
    SNAP_KESSLER_ADJ_CASE(4)
    SNAP_KESSLER_ADJ_CASE(5)
    SNAP_KESSLER_ADJ_CASE(6)
    SNAP_KESSLER_ADJ_CASE(7)
    SNAP_KESSLER_ADJ_CASE(8)
#undef SNAP_KESSLER_ADJ_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_kessler_adj(int dtype, int ntracer, const void* q, void* qb, const KesslerArgs& a,
                       hipStream_t st) {
  return dtype == 0 ? launch_kessler_adj_t<double>(ntracer, static_cast<const double*>(q),
                                                   static_cast<double*>(qb), a, st)
                    : launch_kessler_adj_t<float>(ntracer, static_cast<const float*>(q),
                                                  static_cast<float*>(qb), a, st);
}

template <typename T>
int launch_satadj_t(int ntracer, T* q, const SatAdjArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.ny * a.nz), (unsigned)((a.nx + 255) / 256));
  switch (ntracer) {
#define SNAP_SATADJ_CASE(N)                                                         \
  case N:                                                                           \
    hipLaunchKernelGGL((k_satadj<T, N>), grid, dim3(256), 0, st, q, a);             \
    break;
    SNAP_SATADJ_CASE(2)
    SNAP_SATADJ_CASE(3)
    SNAP_SATADJ_CASE(4)
    SNAP_SATADJ_CASE(5)
    SNAP_SATADJ_CASE(6)
    SNAP_SATADJ_CASE(7)
    SNAP_SATADJ_CASE(8)
#undef SNAP_SATADJ_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_satadj(int dtype, int ntracer, void* q, const SatAdjArgs& a, hipStream_t st) {
  return dtype == 0 ? launch_satadj_t<double>(ntracer, static_cast<double*>(q), a, st)
                    : launch_satadj_t<float>(ntracer, static_cast<float*>(q), a, st);
}

template <typename T>
int launch_satadj_adj_t(int ntracer, const T* q, T* qb, const SatAdjArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.ny * a.nz), (unsigned)((a.nx + 255) / 256));
  switch (ntracer) {
#define SNAP_SATADJ_ADJ_CASE(N)                                                     \
  case N:                                                                           \
    hipLaunchKernelGGL((k_satadj_adj<T, N>), grid, dim3(256), 0, st, q, qb, a);     \
    break;
    SNAP_SATADJ_ADJ_CASE(2)
    SNAP_SATADJ_ADJ_CASE(3)
    SNAP_SATADJ_ADJ_CASE(4)
    SNAP_SATADJ_ADJ_CASE(5)
    SNAP_SATADJ_ADJ_CASE(6)
    SNAP_SATADJ_ADJ_CASE(7)
    SNAP_SATADJ_ADJ_CASE(8)
#undef SNAP_SATADJ_ADJ_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_satadj_adj(int dtype, int ntracer, const void* q, void* qb, const SatAdjArgs& a,
                      hipStream_t st) {
  return dtype == 0 ? launch_satadj_adj_t<double>(ntracer, static_cast<const double*>(q),
                                                  static_cast<double*>(qb), a, st)
                    : launch_satadj_adj_t<float>(ntracer, static_cast<const float*>(q),
                                                 static_cast<float*>(qb), a, st);
}

}  // namespace snap
