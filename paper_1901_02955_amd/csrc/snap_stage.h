// Fused right-hand-side / Runge-Kutta stage kernels.
//
// One launch evaluates the full right-hand side of Sec. 4 (eq. forward) for a
// block of cells and either stores it (rhs mode) or applies one stage of the
// TVD Runge-Kutta step of Sec. 4.3 (stage mode):
//     out = ca * Qn + cb * (Qs + dt * R(Qs)).
// Face states and fluxes never leave the chip: primitive variables of a plane
// of cells and the face values / fluxes of its two in-plane directions are
// staged through LDS, and (3-D) the vertical direction is marched with a
// per-thread register window of five levels.
//
// 3-D kernel: a workgroup owns a TX x TY column tile and a chunk of levels;
//   it walks up the chunk, and per level
//     (P) writes the primitives of the tile and its 3-cell x/y halo to LDS,
//     (R) reconstructs every cell of the tile plus one halo cell on each side
//         in x and in y (WENO5, both faces of the cell),
//     (L) evaluates LMARS at every x and y face of the tile,
//     (D) forms the divergence with the vertical flux difference that the
//         thread's own register window produced, adds gravity, and writes.
// 2-D (x-z) kernel: a workgroup owns a TX x TZ tile of the x-z plane and runs
//   the same P/R/L/D phases once, with z as the second in-plane axis.
#pragma once

#include "snap_device.h"

// Optional scheduling fence between per-variable reconstructions: keeps the
// compiler from interleaving all variables' WENO work (which raises register
// pressure and costs occupancy in double precision).
#ifdef SNAP_SCHED_FENCE
#define SNAP_VAR_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define SNAP_VAR_FENCE() ((void)0)
#endif

namespace snap {

#ifndef SNAP_MAX_PASSES
#define SNAP_MAX_PASSES 8
#endif

struct StageArgs {
  const void* qs;   // padded state whose right-hand side is taken (ghosts filled)
  const void* qn;   // padded Q^n for the stage combination (may alias out); unused if ca == 0
  void* out;        // padded next state (stage mode) or interior rhs (rhs mode)
  int rhs_mode;     // 1: out = R (interior layout); 0: stage combination (padded layout)
  double ca, cb, dt;
  int nx, ny, nz;
  int gy;                  // 3 in 3-D, 0 in 2-D
  long long sy, sz, sv;    // padded strides (elements)
  long long ry, rz, rv;    // interior (rhs) strides
  int tiles_x, tiles_y, nchunk, tz;
  // 3-D only. pass_map = 0: block -> (tile, chunk) through the XCD-aware
  // order, chunk kc covering levels kc*tz .. min(kc*tz + tz, nz) - 1.
  // pass_map = 1 (a launch of exactly one workgroup per compute unit per
  // chunk, all co-resident): chunk kc = blockIdx / tiles, i.e. the dispatch
  // pass, covering levels kb[kc] .. kb[kc+1] - 1; consecutive blocks of a
  // pass go to different XCDs, and the tiles one XCD receives are adjacent.
  int pass_map;
  int kb[SNAP_MAX_PASSES + 1];
  double dxi, dyi, dzi;    // 1 / spacing
  double gamma, gm1, inv_gm1, grav, eps;
  int linear;
  const double* rbar_c;  // nz + 6
  const double* pbar_c;
  const double* rbar_f;  // nz + 1
  const double* pbar_f;
  Mixture mix;           // mixture equation of state (kernels instantiated with MIX)
  Sediment sed;          // sedimentation (3-D: SED kernel instances; 2-D: a kernel of its own)
  // Time step from the device: when smax is set, dt = cfl / (the maximum
  // signal speed whose IEEE bits smax holds, written by the reduction kernel
  // earlier on the stream) and a.dt is unused. When dt_out is set, block 0
  // stores the dt it used there.
  const unsigned long long* smax;
  double cfl;
  double* dt_out;
  // 3-D only. GF_ON: the kernel reads each ghost cell it needs (the x / y
  // halo of its tile, the window levels below 0 and above nz - 1) from the
  // interior cell the ghost fill copies (ghost_src, momentum normal to a
  // reflecting wall negated), so no fill has to precede it; GF_RX / GF_RY /
  // GF_RZ: that axis reflects (else it is periodic).
  int ghost;
  // Next step's time step (kernels that read ghosts in place):
  // with smax_out set, the kernel also reduces the maximum signal speed of its
  // output (the quantity and the arithmetic of the CFL reduction kernel, so the
  // dt formed from it is the same) into *smax_out with atomicMax; with
  // smax_zero set, block 0 clears *smax_zero (a slot that a later launch of
  // the step fills).
  unsigned long long* smax_out;
  unsigned long long* smax_zero;
  // With the time step from the device (smax set): block 0 stores 1 here if
  // that time step is not finite and positive, i.e. the reduced state had a
  // non-finite or non-positive density or pressure somewhere.
  unsigned long long* state_flag;
  // 1: q holds rho - rhobar_k and E - pbar_k / (gamma - 1) (perturbation
  // storage, passive tracers only); 0: the full conserved state.
  int pert;
};

// References of level k for the conversion of the stored state: ra is added
// to the stored density to give rho, rs and ps are subtracted from rho and p
// to give rho' and p'; pe is added to (gamma - 1)(E_stored - K) to give p.
struct LevelRef {
  double ra, rs, ps, pe;
};
__device__ __forceinline__ LevelRef level_ref(int pert, double rbar, double pbar) {
  LevelRef r;
  r.ra = pert ? rbar : 0.0;
  r.rs = pert ? 0.0 : rbar;
  r.ps = pert ? 0.0 : pbar;
  r.pe = pert ? pbar : 0.0;
  return r;
}
enum : int { GF_ON = 1, GF_RX = 2, GF_RY = 4, GF_RZ = 8 };

// The 3-D stage kernels that can read ghosts in place (GF_ON): those without
// tracers. With tracers the extra per-level scalar work pushed some instances
// past an occupancy step, and they keep the fill.
constexpr bool ghosts_in_place(int ntracer) { return ntracer == 0; }

// Kernels that can reduce the signal speed of their output (smax_out).
template <typename T, int NT>
constexpr bool fused_speed() { return ghosts_in_place(NT); }


// The stage's time step (uniform over the launch).
__device__ __forceinline__ double stage_dt(const StageArgs& a) {
  if (a.smax == nullptr) return a.dt;
  return a.cfl / __longlong_as_double(static_cast<long long>(*a.smax));
}

// Block 0 records the time step of the launch where the caller asked for it,
// and raises the state flag if that time step is not finite and positive.
__device__ __forceinline__ void store_stage_dt(const StageArgs& a, double dt) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    if (a.dt_out != nullptr) *a.dt_out = dt;
    if (a.state_flag != nullptr && !(dt > 0.0 && dt <= 1.79769313486231570815e308))
      *a.state_flag = 1ULL;
  }
}

template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return static_cast<double>(v);
}

// Load the NV conserved values of padded element offset `off` and convert them
// to primitives with the level references (rb, pb).
// Conserved -> primitive with the kernel's equation of state: passive tracers,
// or the mixture (MIX) with coefficients mx.
template <int NV, bool MIX>
__device__ __forceinline__ void cons_to_prim_eos(const double (&c)[NV], double ra, double rb,
                                                 double pb, double gm1, const Mixture& mx,
                                                 double (&x)[NV]) {
  if constexpr (MIX)
    cons_to_prim_mix<NV>(c, rb, pb, gm1, mx, x);   // full storage only (ra = 0)
  else
    cons_to_prim<NV>(c, ra, rb, pb, gm1, x);
}

// Single-precision storage with passive tracers: the velocities, kinetic
// energy and tracer fractions in single precision, where nothing cancels, and
// only the two differences that do, rho - rhobar and (gamma - 1)(E - K) -
// pbar, in double precision (one rounding each, then to single precision).
// The reciprocal of rho is the hardware estimate (1 ulp).
template <int NV>
__device__ __forceinline__ void cons_to_prim_sp(const float (&c)[NV], double ra, double rb,
                                                double pb, double gm1, float (&x)[NV]) {
  const float inv = __builtin_amdgcn_rcpf(c[0] + static_cast<float>(ra));
  const float u = c[1] * inv, v = c[2] * inv, w = c[3] * inv;
  const float K = 0.5f * fmaf(c[3], w, fmaf(c[2], v, c[1] * u));
  x[0] = static_cast<float>(static_cast<double>(c[0]) - rb);
  x[1] = u;
  x[2] = v;
  x[3] = w;
  x[4] = static_cast<float>(fma(gm1, static_cast<double>(c[4]) - static_cast<double>(K), -pb));
#pragma unroll
  for (int t = 5; t < NV; ++t) x[t] = c[t] * inv;
}

template <typename T, int NV, bool MIX = false>
__device__ __forceinline__ void load_prim(const T* __restrict__ q, long long off, long long sv,
                                          const LevelRef& lr, double gm1, const Mixture& mx,
                                          T (&x)[NV]) {
  if constexpr (sizeof(T) == 4 && !MIX) {
    float c[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = q[off + v * sv];
    cons_to_prim_sp<NV>(c, lr.ra, lr.rs, lr.ps, gm1, x);
  } else {
    double c[NV], xd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = to_d(q[off + v * sv]);
    cons_to_prim_eos<NV, MIX>(c, lr.ra, lr.rs, lr.ps, gm1, mx, xd);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = static_cast<T>(xd[v]);
  }
}

// passive tracers
template <typename T, int NV>
__device__ __forceinline__ void load_prim(const T* __restrict__ q, long long off, long long sv,
                                          const LevelRef& lr, double gm1, T (&x)[NV]) {
  if constexpr (sizeof(T) == 4) {
    float c[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = q[off + v * sv];
    cons_to_prim_sp<NV>(c, lr.ra, lr.rs, lr.ps, gm1, x);
  } else {
    double c[NV], xd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = to_d(q[off + v * sv]);
    cons_to_prim<NV>(c, lr.ra, lr.rs, lr.ps, gm1, xd);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = static_cast<T>(xd[v]);
  }
}

// The factor by which riemann_flux scales the face flux: the passive LMARS
// returns twice the flux (lmars_flux), the others the flux itself. The flux
// differences are multiplied by the inverse spacing over this factor (a power
// of two, so the scaled spacing is exact).
template <bool MIX, bool HLLC>
constexpr double flux_scale() {
  return (!MIX && !HLLC) ? 2.0 : 1.0;
}

// Face flux of the kernel's Riemann solver (LMARS, or HLLC with passive
// tracers) and equation of state, times flux_scale<MIX, HLLC>().
template <typename T, int NV, bool MIX, bool HLLC>
__device__ __forceinline__ void riemann_flux(const T (&xl)[NV], const T (&xr)[NV], int nrm,
                                             T rref, T pref, T gamma, T inv_gm1, T gm1,
                                             const Mixture& mx, T (&f)[NV]) {
  static_assert(!(MIX && HLLC), "HLLC takes passive tracers");
  if constexpr (HLLC)
    hllc_flux<T, NV>(xl, xr, nrm, rref, pref, gamma, inv_gm1, f);
  else if constexpr (MIX)
    lmars_flux_mix<T, NV>(xl, xr, nrm, rref, pref, gm1, mx, f);
  else
    lmars_flux<T, NV>(xl, xr, nrm, rref, pref, gamma, inv_gm1, f);
}

// Output of one interior cell: either R itself or the stage combination.
template <typename T, int NV>
__device__ __forceinline__ void write_cell(const StageArgs& a, const T* __restrict__ qs,
                                           long long poff, long long roff, const T (&R)[NV]) {
  if (a.rhs_mode) {
    T* __restrict__ o = static_cast<T*>(a.out);
#pragma unroll
    for (int v = 0; v < NV; ++v) o[roff + v * a.rv] = R[v];
    return;
  }
  const T dt = static_cast<T>(stage_dt(a)), ca = static_cast<T>(a.ca), cb = static_cast<T>(a.cb);
  T* o = static_cast<T*>(a.out);
  const T* qn = static_cast<const T*>(a.qn);
  if (a.ca != 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T t = qs[poff + v * a.sv] + dt * R[v];
      o[poff + v * a.sv] = ca * qn[poff + v * a.sv] + cb * t;
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T t = qs[poff + v * a.sv] + dt * R[v];
      o[poff + v * a.sv] = cb * t;
    }
  }
}

// ---------------------------------------------------------------------------
// LDS plane shared by both kernels: primitives with a 3-cell halo and, per
// in-plane axis, one value per face (first the left face state, then, after
// the LMARS phase, the flux). The right face state of each face stays in the
// registers of the thread that reconstructed it; the items beyond the RREG
// rounds, reconstructed one (cell, variable) pair at a time, park it in QS.
//
// Work items of the reconstruction and LMARS phases (one list; within the
// RREG rounds the same thread takes an item in both):
//   x items: cells ii = -1 .. TX along each row jj = 0 .. TY-1;
//   second-axis items: cells jj = -1 .. TY along each column ii = 0 .. TX-1.
// Item (cell c) writes the left state of face c+1 and keeps the right state
// of face c; in the LMARS phase it evaluates face c (for c >= 0).
// ---------------------------------------------------------------------------
template <int TX, int TY>
struct PlaneItems {
  static constexpr int NTHR = TX * TY;
  static constexpr int NRX = (TX + 2) * TY;
  static constexpr int NRS = TX * (TY + 2);
  static constexpr int NR = NRX + NRS;
  static constexpr int ROUNDS = (NR + NTHR - 1) / NTHR;
#ifndef SNAP_RREG
#define SNAP_RREG 2
#endif
  static constexpr int RREG = ROUNDS < SNAP_RREG ? ROUNDS : SNAP_RREG;
  static constexpr int NSPILL = NR - RREG * NTHR > 0 ? NR - RREG * NTHR : 1;
};

template <typename T, int NV, int TX, int TY>
struct Plane {
  T P[NV][TY + 6][TX + 6];
  T FX[NV][TY][TX + 1];
  T FY[NV][TY + 1][TX];
  T QS[PlaneItems<TX, TY>::NSPILL][NV];
};

// Thread index used for item lists: the waves of a workgroup take turns at
// the rounds that not every wave gets (e.g. 576 items over 4 waves), rotated
// by block so that co-resident workgroups put the extra round on different
// SIMDs.
template <int NTHR>
__device__ __forceinline__ int item_thread() {
  if constexpr (NTHR % 64 == 0 && NTHR >= 128)
    return (threadIdx.x + 64 * (blockIdx.x % (NTHR / 64))) % NTHR;
  else
    return threadIdx.x;
}

// Decode item `it` into (axis, ii, jj); returns false if the cell lies outside
// the active w x h part of a ragged tile.
template <int TX, int TY>
__device__ __forceinline__ bool plane_item(int it, int w, int h, bool& xaxis, int& ii, int& jj) {
  using I = PlaneItems<TX, TY>;
  if (it < I::NRX) {
    xaxis = true;
    ii = it % (TX + 2) - 1;
    jj = it / (TX + 2);
    return ii <= w && jj < h;
  }
  const int r = it - I::NRX;
  xaxis = false;
  ii = r % TX;
  jj = r / TX - 1;
  return ii < w && jj <= h;
}

// Phase R: WENO5 of every item cell; left states to LDS, right states kept
// (in registers for the RREG rounds, in QS for the items beyond them).
// An x item reads a row of the plane (stride 1), a second-axis item a column
// (stride TX + 6), so one code path serves both. With RPF the five stencil
// values of variable v + 1 are read from LDS before variable v is
// reconstructed: the LDS latency then overlaps that reconstruction instead of
// stalling the wave at the start of every variable. RPF is off where those
// five live values would push the kernel past an occupancy step.
template <typename T, int NV>
constexpr bool reconstruct_prefetch() {
  // single precision with 1 or 8 tracers: 167 -> 178 and 256 -> 257 registers
  return !(sizeof(T) == 4 && (NV == 6 || NV == 13));
}

// SPLIT: the items beyond the RREG rounds (64 of the 576 of a 16 x 16 tile)
// are split by variable, one (cell, variable) pair per thread and pass, so
// that every wave takes a share instead of one wave reconstructing all their
// variables while the others wait at the barrier. Without SPLIT they are a
// last round of whole items, which needs fewer registers: the callers keep
// that form where the split would cost a wave per SIMD or add spills.
template <typename T, int NV, int TX, int TY, bool SPLIT = true>
__device__ __forceinline__ void phase_reconstruct(Plane<T, NV, TX, TY>& S, int w, int h, T eps,
                                                  bool linear,
                                                  T (&QP)[PlaneItems<TX, TY>::RREG][NV]) {
  using I = PlaneItems<TX, TY>;
  constexpr bool RPF = reconstruct_prefetch<T, NV>();
  constexpr int PV = (TY + 6) * (TX + 6);   // plane stride between variables
  constexpr int FXV = TY * (TX + 1), FYV = (TY + 1) * TX;
  constexpr int NSP = I::NR - I::RREG * I::NTHR;   // cells left after the RREG rounds
  if constexpr (SPLIT && NSP > 0) {
    constexpr int NSUB = NSP * NV;
    const int t0 = item_thread<I::NTHR>();
#pragma unroll
    for (int m = 0; m < (NSUB + I::NTHR - 1) / I::NTHR; ++m) {
      const int sub = t0 + m * I::NTHR;
      const int v = sub / NSP, c = sub - v * NSP;
      const int it = I::RREG * I::NTHR + c;
      bool xa;
      int ii, jj;
      if (sub < NSUB && plane_item<TX, TY>(it, w, h, xa, ii, jj)) {
        const int st = xa ? 1 : TX + 6;
        const T* src = (xa ? &S.P[0][jj + 3][ii + 1] : &S.P[0][jj + 1][ii + 3]) + v * PV;
        T cur[5];
#pragma unroll
        for (int mm = 0; mm < 5; ++mm) cur[mm] = src[mm * st];
        T qm, qp;
        weno5_cell<T>(cur[0], cur[1], cur[2], cur[3], cur[4], eps, linear, qm, qp);
        if (xa ? ii < w : jj < h) {
          if (xa)
            S.FX[v][jj][ii + 1] = qm;
          else
            S.FY[v][jj + 1][ii] = qm;
        }
        S.QS[c][v] = qp;
      }
    }
  }
  constexpr int NROUND = SPLIT ? I::RREG : I::ROUNDS;
#pragma unroll
  for (int r = 0; r < NROUND; ++r) {
    const int it = item_thread<I::NTHR>() + r * I::NTHR;
    bool xa;
    int ii, jj;
    if (it < I::NR && plane_item<TX, TY>(it, w, h, xa, ii, jj)) {
      const int st = xa ? 1 : TX + 6;
      const T* src = xa ? &S.P[0][jj + 3][ii + 1] : &S.P[0][jj + 1][ii + 3];
      T* dst = xa ? &S.FX[0][jj][ii + 1] : &S.FY[0][jj + 1][ii];
      const int dv = xa ? FXV : FYV;
      const bool put = xa ? ii < w : jj < h;
      T qp[NV];
      T cur[5];
      if constexpr (RPF) {
#pragma unroll
        for (int m = 0; m < 5; ++m) cur[m] = src[m * st];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T nxt[5];
        if constexpr (RPF) {
          if (v + 1 < NV) {
#pragma unroll
            for (int m = 0; m < 5; ++m) nxt[m] = src[(v + 1) * PV + m * st];
          }
        } else {
#pragma unroll
          for (int m = 0; m < 5; ++m) cur[m] = src[v * PV + m * st];
        }
        T qm;
        weno5_cell<T>(cur[0], cur[1], cur[2], cur[3], cur[4], eps, linear, qm, qp[v]);
        if (put) dst[v * dv] = qm;
        SNAP_VAR_FENCE();
        if constexpr (RPF) {
          if (v + 1 < NV) {
#pragma unroll
            for (int m = 0; m < 5; ++m) cur[m] = nxt[m];
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (r < I::RREG)
          QP[r < I::RREG ? r : 0][v] = qp[v];
        else
          S.QS[it - I::RREG * I::NTHR][v] = qp[v];
      }
    }
  }
}

// Phase L: LMARS at every face of the tile, by the item that holds its right
// state. x faces use the reference of their row (xref); second-axis faces use
// sref(face index). SNRM is the index of the second axis's velocity; the flux
// is called in two branches, each with a constant normal, so that picking the
// normal velocity and adding p* need no selects over the velocity components.
template <typename T, int NV, int TX, int TY, int SNRM, bool MIX, bool HLLC, typename XRef,
          typename SRef>
__device__ __forceinline__ void phase_lmars(Plane<T, NV, TX, TY>& S, int w, int h,
                                            T gamma, T inv_gm1, T gm1, const Mixture& mx,
                                            XRef xref, SRef sref,
                                            const T (&QP)[PlaneItems<TX, TY>::RREG][NV]) {
  using I = PlaneItems<TX, TY>;
#pragma unroll
  for (int r = 0; r < I::ROUNDS; ++r) {
    const int it = item_thread<I::NTHR>() + r * I::NTHR;
    bool xa;
    int ii, jj;
    if (it < I::NR && plane_item<TX, TY>(it, w, h, xa, ii, jj) && ii >= 0 && jj >= 0) {
      T xl[NV], xr[NV], f[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        xr[v] = r < I::RREG ? QP[r < I::RREG ? r : 0][v] : S.QS[it - I::RREG * I::NTHR][v];
        xl[v] = xa ? S.FX[v][jj][ii] : S.FY[v][jj][ii];
      }
      T rr, pr;
      if (xa) {
        xref(jj, rr, pr);
        riemann_flux<T, NV, MIX, HLLC>(xl, xr, 1, rr, pr, gamma, inv_gm1, gm1, mx, f);
      } else {
        sref(jj, rr, pr);
        riemann_flux<T, NV, MIX, HLLC>(xl, xr, SNRM, rr, pr, gamma, inv_gm1, gm1, mx, f);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (xa)
          S.FX[v][jj][ii] = f[v];
        else
          S.FY[v][jj][ii] = f[v];
      }
    }
  }
}

// Halo item it of the plane: 6 cells beyond each x edge of every row, then 6
// beyond each second-axis edge of every column. Returns false outside the
// active part of a ragged tile.
template <int TX, int TY>
__device__ __forceinline__ bool halo_item(int it, int w, int h, int& ii, int& jj) {
  // selects rather than two branches that each write one of ii / jj: the
  // compiler would merge those writes into one store through a selected
  // address and keep ii, jj in scratch memory
  const bool xs = it < 6 * TY;   // x halo (columns left / right of the tile)
  const int r = xs ? it : it - 6 * TY;
  const int m = r % 6, q = r / 6;
  const int e = m < 3 ? m - 3 : (xs ? w : h) + m - 3;
  ii = xs ? e : q;
  jj = xs ? q : e;
  return q < (xs ? h : w);
}

// The 3-D kernels that split the reconstruction's last items by variable
// (phase_reconstruct): not those with the sedimentation terms, which are held
// to two waves per SIMD in single precision (with six tracers the split took
// the spilled registers from 3 to 11).
template <typename T, int NT, bool MIX, bool SED>
constexpr bool split_reconstruct() {
  return !SED;
}

// ---------------------------------------------------------------------------
// 3-D kernel
// ---------------------------------------------------------------------------
#ifndef SNAP_STAGE3D_WAVES_PER_EU
#define SNAP_STAGE3D_WAVES_PER_EU 1
#endif

template <typename T, int NV>
__device__ __forceinline__ void load_cons(const T* __restrict__ q, long long off, long long sv,
                                          T (&c)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = q[off + v * sv];
}

template <typename T, int NV, bool MIX>
__device__ __forceinline__ void cons_to_prim_t(const T (&c)[NV], const LevelRef& lr, double gm1,
                                               const Mixture& mx, T (&x)[NV]) {
  if constexpr (sizeof(T) == 4 && !MIX) {
    cons_to_prim_sp<NV>(c, lr.ra, lr.rs, lr.ps, gm1, x);
    return;
  }
  double cd[NV], xd[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) cd[v] = static_cast<double>(c[v]);
  cons_to_prim_eos<NV, MIX>(cd, lr.ra, lr.rs, lr.ps, gm1, mx, xd);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = static_cast<T>(xd[v]);
}

// SED (mixture with falling condensates): the sedimentation terms of Sec. 2
// (the fall fluxes of mass, momentum and energy through the z faces and the
// frictional heating, sediment_cell) are added to the right-hand side in phase
// D from the window's levels s-1, s, s+1; these instances load nothing a
// level ahead, which makes room for that work in the registers.
// The sedimentation instances in single precision are held to two waves per
// SIMD, and so are the single-precision mixture with six or seven tracers and
// the double-precision sedimentation instance with one tracer (unheld they
// take 258 to 262 registers); the other kernels with up to eight tracers in
// single precision and one in double precision reach it unaided.
template <typename T, int NT, bool MIX, bool SED>
constexpr int stage3d_min_waves() {
  if constexpr (sizeof(T) == 4)
    return (SED || (MIX && (NT == 6 || NT == 7))) ? 2 : SNAP_STAGE3D_WAVES_PER_EU;
  else
    return (SED && NT == 1) ? 2 : SNAP_STAGE3D_WAVES_PER_EU;
}

template <typename T, int NT, int TX, int TY, bool MIX = false, bool HLLC = false,
          bool SED = false>
__global__ void __launch_bounds__(TX* TY, (stage3d_min_waves<T, NT, MIX, SED>()))
    k_stage3d(StageArgs a) {
  constexpr int NV = 5 + NT;
  constexpr bool GF = ghosts_in_place(NT);
  static_assert(!SED || (MIX && NT > 0 && !HLLC), "sedimentation needs the mixture");
  using I = PlaneItems<TX, TY>;
  constexpr int NHALO = 6 * (TX + TY);
  constexpr int HR = (NHALO + I::NTHR - 1) / I::NTHR;   // halo items per thread
  // Load the next level's halo, window and stage-combination values a level
  // ahead only where the extra 4 NV live values still leave room for two
  // waves per SIMD (256 registers); with more variables each value is loaded
  // where it is used.
  constexpr bool PF = !SED && (sizeof(T) == 4 ? NV <= 11 : NV <= 5);
  __shared__ Plane<T, NV, TX, TY> S;
  const T* __restrict__ qs = static_cast<const T*>(a.qs);

  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  int tx, ty, k0, k1;
  if (a.pass_map) {
    const int tiles = a.tiles_x * a.tiles_y;
    const int kc = blockIdx.x / tiles;
    const int r = blockIdx.x - kc * tiles;
    const int t = (r % 8) * (tiles / 8) + r / 8;
    tx = t % a.tiles_x;
    ty = t / a.tiles_x;
    k0 = a.kb[kc];
    k1 = a.kb[kc + 1];
  } else {
    const int L = xcd_logical_block(blockIdx.x, gridDim.x);
    tx = L % a.tiles_x;
    const int rr_ = L / a.tiles_x;
    ty = rr_ % a.tiles_y;
    const int kc = rr_ / a.tiles_y;
    k0 = kc * a.tz;
    k1 = min(k0 + a.tz, a.nz);
  }
  const int i0 = tx * TX, j0 = ty * TY;
  const int w = min(TX, a.nx - i0), h = min(TY, a.ny - j0);
  const bool act = ti < w && tj < h;
  const T eps = static_cast<T>(a.eps), gamma = static_cast<T>(a.gamma);
  const T inv_gm1 = static_cast<T>(a.inv_gm1), gm1t = static_cast<T>(a.gm1);
  const T dzi = static_cast<T>(a.dzi);   // the sedimentation terms' own differences
  // inverse spacings for the flux differences (the fluxes carry flux_scale)
  constexpr double FSI = 1.0 / flux_scale<MIX, HLLC>();
  const T fdx = static_cast<T>(a.dxi * FSI), fdy = static_cast<T>(a.dyi * FSI);
  const T fdz = static_cast<T>(a.dzi * FSI);
  const bool linear = a.linear != 0;
  // read before any store: the stores of the level loop could alias *a.smax,
  // and a load inside the loop would be repeated at every level
  const double dtd = stage_dt(a);
  store_stage_dt(a, dtd);
  constexpr bool FS = fused_speed<T, NT>();
  if constexpr (FS) {
    if (a.smax_zero != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.smax_zero = 0ULL;
  }
  // running maximum (IEEE bits) of the output's signal speed: one LDS slot per
  // thread, which keeps it out of the registers the level loop needs
  __shared__ unsigned long long smx_lds[FS ? TX * TY : 1];
  if constexpr (FS) smx_lds[tid] = 0ULL;
  const bool combine = a.rhs_mode == 0;
  const bool use_qn = combine && a.ca != 0.0;
  const T* qn = static_cast<const T*>(a.qn);

  // padded offset of (i, j, k) with interior coordinates (k may be a ghost level)
  auto poff = [&](int i, int j, int k) -> long long {
    return (long long)(k + NG) * a.sz + (long long)(j + NG) * a.sy + (i + NG);
  };
  const int ic = i0 + (act ? ti : 0), jc = j0 + (act ? tj : 0);
  const long long col = poff(ic, jc, 0) - (long long)NG * a.sz;   // offset of level -3

  // halo items of this thread (fixed across levels) and their column offsets;
  // with ghost_free a halo cell beyond the domain is read at the interior cell
  // the fill would copy (its momentum normal to a reflecting wall is negated
  // where it is planed)
  int hii[HR], hjj[HR];
  bool hok[HR];
  long long hoff[HR];
#pragma unroll
  for (int r = 0; r < HR; ++r) {
    const int it = item_thread<I::NTHR>() + r * I::NTHR;
    hok[r] = it < NHALO && halo_item<TX, TY>(it, w, h, hii[r], hjj[r]);
    int gi = i0 + hii[r], gj = j0 + hjj[r];
    if (GF && (a.ghost & GF_ON) && hok[r]) {
      bool fx, fy;
      gi = ghost_src(gi, a.nx, (a.ghost & GF_RX) ? 1 : 0, fx);
      gj = ghost_src(gj, a.ny, (a.ghost & GF_RY) ? 1 : 0, fy);
    }
    hoff[r] = hok[r] ? poff(gi, gj, 0) - (long long)NG * a.sz : 0;
  }
  auto lev = [&](int k) -> long long { return (long long)(k + NG) * a.sz; };
  // level read for window level k (uniform): k itself, or with GF_ON the
  // level a z ghost copies; zf: rho w changes sign (mirror at a z wall)
  auto zsrc = [&](int k, bool& zf) -> int {
    zf = false;
    if (GF && (a.ghost & GF_ON) && (k < 0 || k >= a.nz))
      return ghost_src(k, a.nz, (a.ghost & GF_RZ) ? 1 : 0, zf);
    return k;
  };

  T W[5][NV];     // primitives of levels s-1 .. s+3 (own column)
  T qmc[NV];      // left state at the vertical face above the current level
  T fzc[NV];      // vertical flux at the lower face of the current level
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    qmc[v] = T(0);
    fzc[v] = T(0);
  }
  if (act) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int k = k0 - 3 + l;
      bool zf;
      T c[NV];
      load_cons<T, NV>(qs, col + lev(zsrc(k, zf)), a.sv, c);
      if (zf) c[3] = -c[3];
      cons_to_prim_t<T, NV, MIX>(c, level_ref(a.pert, a.rbar_c[k + NG], a.pbar_c[k + NG]), a.gm1,
                                 a.mix, W[l]);
    }
  }
  // prefetched raw conserved values: halo cells of the next level to be
  // planed, the window's next level, and this level's own Qs / Qn
  T hc[HR][NV];
  if constexpr (PF) {
#pragma unroll
    for (int r = 0; r < HR; ++r)
      if (hok[r]) load_cons<T, NV>(qs, hoff[r] + lev(k0), a.sv, hc[r]);
  }
  // this level's own Qs (and Qn): the stage combination and the gravity work
  auto load_own = [&](int s, T (&qsc)[NV], T (&qnc)[NV]) {
    if (combine) {
      load_cons<T, NV>(qs, col + lev(s), a.sv, qsc);
      if (use_qn) load_cons<T, NV>(qn, col + lev(s), a.sv, qnc);
    } else {
      qsc[3] = qs[col + lev(s) + 3 * a.sv];
    }
  };

  T QP[I::RREG][NV];
  for (int s = k0 - 2; s < k1; ++s) {
    T wc[NV], qsc[NV], qnc[NV];
    bool wzf;
    const int wsrc = zsrc(s + 3, wzf);
    if constexpr (PF) {
      if (act) {
        load_cons<T, NV>(qs, col + lev(wsrc), a.sv, wc);
        if (s >= k0) load_own(s, qsc, qnc);
      }
    }
    if (s >= k0) {
      // ---- (P) primitives of level s: own cell from the window, halo prefetched
      const double rbs = a.rbar_c[s + NG], pbs = a.pbar_c[s + NG];
      const LevelRef lrs = level_ref(a.pert, rbs, pbs);
      if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) S.P[v][tj + 3][ti + 3] = W[1][v];
      }
#pragma unroll
      for (int r = 0; r < HR; ++r) {
        if (hok[r]) {
          T x[NV];
          if constexpr (!PF) load_cons<T, NV>(qs, hoff[r] + lev(s), a.sv, hc[r]);
          if (GF && (a.ghost & GF_ON) && (a.ghost & (GF_RX | GF_RY))) {
            const int gi = i0 + hii[r], gj = j0 + hjj[r];
            if ((a.ghost & GF_RX) && (gi < 0 || gi >= a.nx)) hc[r][1] = -hc[r][1];
            if ((a.ghost & GF_RY) && (gj < 0 || gj >= a.ny)) hc[r][2] = -hc[r][2];
          }
          cons_to_prim_t<T, NV, MIX>(hc[r], lrs, a.gm1, a.mix, x);
#pragma unroll
          for (int v = 0; v < NV; ++v) S.P[v][hjj[r] + 3][hii[r] + 3] = x[v];
          if constexpr (PF) {
            if (s + 1 < k1) load_cons<T, NV>(qs, hoff[r] + lev(s + 1), a.sv, hc[r]);
          }
        }
      }
      __syncthreads();
      // ---- (R) WENO5 in x and y ---------------------------------------------
      phase_reconstruct<T, NV, TX, TY, split_reconstruct<T, NT, MIX, SED>()>(S, w, h, eps,
                                                                            linear, QP);
      __syncthreads();
      // ---- (L) LMARS at x and y faces (level references) ---------------------
      const T rbT = static_cast<T>(rbs), pbT = static_cast<T>(pbs);
      auto levref = [&](int, T& r, T& p) {
        r = rbT;
        p = pbT;
      };
      phase_lmars<T, NV, TX, TY, 2, MIX, HLLC>(S, w, h, gamma, inv_gm1, gm1t, a.mix, levref,
                                            levref, QP);
      __syncthreads();
    }
    // ---- vertical direction, own column: face s+1/2 (z-face index s+1) -------
    T dfz[NV];
    if (act) {
      if constexpr (!PF) load_cons<T, NV>(qs, col + lev(wsrc), a.sv, wc);
      if (wzf) wc[3] = -wc[3];
      cons_to_prim_t<T, NV, MIX>(wc, level_ref(a.pert, a.rbar_c[s + 3 + NG], a.pbar_c[s + 3 + NG]),
                                 a.gm1, a.mix, W[4]);
      T qmn[NV], qpn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        weno5_cell<T>(W[0][v], W[1][v], W[2][v], W[3][v], W[4][v], eps, linear, qmn[v], qpn[v]);
        SNAP_VAR_FENCE();
      }
      if (s >= k0 - 1) {
        T fz[NV];
        riemann_flux<T, NV, MIX, HLLC>(qmc, qpn, 3, static_cast<T>(a.rbar_f[s + 1]),
                                       static_cast<T>(a.pbar_f[s + 1]), gamma, inv_gm1, gm1t,
                                       a.mix, fz);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          dfz[v] = fz[v] - fzc[v];
          fzc[v] = fz[v];
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) qmc[v] = qmn[v];
    }
    // ---- (D) divergence, gravity, output -------------------------------------
    if (s >= k0 && act) {
      if constexpr (!PF) load_own(s, qsc, qnc);
      T R[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T r = -((S.FX[v][tj][ti + 1] - S.FX[v][tj][ti]) * fdx);
        r = r - (S.FY[v][tj + 1][ti] - S.FY[v][tj][ti]) * fdy;
        R[v] = r - dfz[v] * fdz;
      }
      const T grav = static_cast<T>(a.grav);
      R[3] = R[3] - grav * W[1][0];
      R[4] = R[4] - grav * qsc[3];
      if constexpr (SED) {
        const bool wall_lo = a.sed.closed_z && s == 0, wall_up = a.sed.closed_z && s == a.nz - 1;
        sediment_cell<T, NV>(W[0], W[1], W[2], static_cast<T>(a.rbar_c[s - 1 + NG]),
                             static_cast<T>(a.pbar_c[s - 1 + NG]), static_cast<T>(a.rbar_c[s + NG]),
                             static_cast<T>(a.pbar_c[s + NG]), static_cast<T>(a.rbar_c[s + 1 + NG]),
                             static_cast<T>(a.pbar_c[s + 1 + NG]), wall_lo, wall_up, a.mix, a.sed,
                             dzi, grav, R);
      }
      const long long po = col + lev(s);
      if (!combine) {
        T* __restrict__ o = static_cast<T*>(a.out);
        const long long ro = (long long)s * a.rz + (long long)jc * a.ry + ic;
#pragma unroll
        for (int v = 0; v < NV; ++v) o[ro + v * a.rv] = R[v];
      } else {
        const T dt = static_cast<T>(dtd), ca = static_cast<T>(a.ca), cb = static_cast<T>(a.cb);
        T* o = static_cast<T*>(a.out);
        T ov[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T t = qsc[v] + dt * R[v];
          ov[v] = use_qn ? ca * qnc[v] + cb * t : cb * t;
          o[po + v * a.sv] = ov[v];
        }
        if constexpr (FS) {
          if (a.smax_out != nullptr) {
            // sum_d (|u_d| + c) / dx_d of the new state (times 1 / dx_d), in the CFL kernel's
            // order and operations (no contraction)
#pragma clang fp contract(off)
            // (perturbation storage: rho and p with the level references added back)
            const double rbo = a.pert ? a.rbar_c[s + NG] : 0.0;
            const double pbo = a.pert ? a.pbar_c[s + NG] : 0.0;
            const double rho = static_cast<double>(ov[0]) + rbo, mx = ov[1], my = ov[2], mz = ov[3];
            const double E = ov[4];
            const double inv = 1.0 / rho;
            const double u = mx * inv, v = my * inv, w = mz * inv;
            const double K = 0.5 * ((mx * u + my * v) + mz * w);
            const double p = a.gm1 * (E - K) + pbo;
            const double cs = sqrt(a.gamma * p / rho);
            double sp = (fabs(u) + cs) * a.dxi;
            sp = sp + (fabs(v) + cs) * a.dyi;
            sp = sp + (fabs(w) + cs) * a.dzi;
            if (!(rho > 0.0) || !(p > 0.0)) sp = __builtin_nan("");
            const unsigned long long sb = (unsigned long long)__double_as_longlong(sp);
            const unsigned long long cur = smx_lds[tid];
            smx_lds[tid] = sb > cur ? sb : cur;
          }
        }
      }
    }
    // shift the window
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
      for (int v = 0; v < NV; ++v) W[l][v] = W[l + 1][v];
  }
  if constexpr (FS) {
    if (a.smax_out != nullptr) {
      unsigned long long smx = smx_lds[tid];
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o2 = __shfl_xor(smx, off, 64);
        smx = o2 > smx ? o2 : smx;
      }
      if ((threadIdx.x & 63) == 0) atomicMax(a.smax_out, smx);
    }
  }
}

// ---------------------------------------------------------------------------
// 2-D (x-z) tile: TX x TZ tile number L of the plane, z is the second in-plane
// axis. Shared by the single-domain kernel and the batched (ensemble) kernel.
// ---------------------------------------------------------------------------
template <typename T, int NT, int TX, int TZ, bool MIX = false, bool HLLC = false>
__device__ __forceinline__ void stage2d_tile(const StageArgs& a, int L,
                                             Plane<T, 5 + NT, TX, TZ>& S) {
  constexpr int NV = 5 + NT;
  using I = PlaneItems<TX, TZ>;
  const T* __restrict__ qs = static_cast<const T*>(a.qs);

  const int tid = threadIdx.x;
  const int ti = tid % TX, tk = tid / TX;
  const int tx = L % a.tiles_x;
  const int tzi = L / a.tiles_x;
  const int i0 = tx * TX, k0 = tzi * TZ;
  const int w = min(TX, a.nx - i0), h = min(TZ, a.nz - k0);
  const bool act = ti < w && tk < h;
  const T eps = static_cast<T>(a.eps), gamma = static_cast<T>(a.gamma);
  const T inv_gm1 = static_cast<T>(a.inv_gm1), gm1t = static_cast<T>(a.gm1);
  // inverse spacings for the flux differences (the fluxes carry flux_scale)
  constexpr double FSI = 1.0 / flux_scale<MIX, HLLC>();
  const T fdx = static_cast<T>(a.dxi * FSI), fdz = static_cast<T>(a.dzi * FSI);
  const bool linear = a.linear != 0;

  auto poff = [&](int i, int k) -> long long { return (long long)(k + NG) * a.sz + (i + NG); };

  // ---- (P) primitives of the tile and its halo --------------------------------
  if (act) {
    const int k = k0 + tk;
    T x[NV];
    load_prim<T, NV, MIX>(qs, poff(i0 + ti, k), a.sv,
                          level_ref(a.pert, a.rbar_c[k + NG], a.pbar_c[k + NG]), a.gm1, a.mix, x);
#pragma unroll
    for (int v = 0; v < NV; ++v) S.P[v][tk + 3][ti + 3] = x[v];
  }
  for (int it = item_thread<I::NTHR>(); it < 6 * (TX + TZ); it += I::NTHR) {
    int ii, kk;
    if (halo_item<TX, TZ>(it, w, h, ii, kk)) {
      const int k = k0 + kk;
      T x[NV];
      load_prim<T, NV, MIX>(qs, poff(i0 + ii, k), a.sv,
                            level_ref(a.pert, a.rbar_c[k + NG], a.pbar_c[k + NG]), a.gm1, a.mix, x);
#pragma unroll
      for (int v = 0; v < NV; ++v) S.P[v][kk + 3][ii + 3] = x[v];
    }
  }
  __syncthreads();
  T QP[I::RREG][NV];
  phase_reconstruct<T, NV, TX, TZ>(S, w, h, eps, linear, QP);
  __syncthreads();
  auto xref = [&](int kk, T& r, T& p) {
    r = static_cast<T>(a.rbar_c[k0 + kk + NG]);
    p = static_cast<T>(a.pbar_c[k0 + kk + NG]);
  };
  auto zref = [&](int fk, T& r, T& p) {
    r = static_cast<T>(a.rbar_f[k0 + fk]);
    p = static_cast<T>(a.pbar_f[k0 + fk]);
  };
  phase_lmars<T, NV, TX, TZ, 3, MIX, HLLC>(S, w, h, gamma, inv_gm1, gm1t, a.mix, xref, zref, QP);
  __syncthreads();
  if (act) {
    T R[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T r = -((S.FX[v][tk][ti + 1] - S.FX[v][tk][ti]) * fdx);
      R[v] = r - (S.FY[v][tk + 1][ti] - S.FY[v][tk][ti]) * fdz;
    }
    const int i = i0 + ti, k = k0 + tk;
    const long long po = poff(i, k);
    const T grav = static_cast<T>(a.grav);
    R[3] = R[3] - grav * S.P[0][tk + 3][ti + 3];
    R[4] = R[4] - grav * qs[po + 3 * a.sv];
    const long long ro = (long long)k * a.rz + i;
    write_cell<T, NV>(a, qs, po, ro, R);
  }
}

template <typename T, int NT, int TX, int TZ, bool MIX = false, bool HLLC = false>
__global__ void __launch_bounds__(TX* TZ) k_stage2d(StageArgs a) {
  __shared__ Plane<T, 5 + NT, TX, TZ> S;
  store_stage_dt(a, stage_dt(a));
  stage2d_tile<T, NT, TX, TZ, MIX, HLLC>(a, xcd_logical_block(blockIdx.x, gridDim.x), S);
}

// Ensemble of 2-D domains in one persistent launch: work item w is tile
// w - first[m] of member m (first[m] <= w < first[m+1]); every block walks the
// items w = blockIdx.x, blockIdx.x + gridDim.x, ... A barrier closes every tile:
// its last phase still reads the primitive plane (density perturbation for the
// gravity source) that the next tile's first phase overwrites.
template <typename T, int NT, int TX, int TZ, bool MIX = false, bool HLLC = false>
__global__ void __launch_bounds__(TX* TZ) k_stage2d_batched(const StageArgs* __restrict__ descs,
                                                            const int* __restrict__ first, int n) {
  __shared__ Plane<T, 5 + NT, TX, TZ> S;
  const int total = first[n];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int lo = 0, hi = n;   // first[lo] <= w < first[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (first[mid] <= w)
        lo = mid;
      else
        hi = mid;
    }
    const StageArgs a = descs[lo];
    stage2d_tile<T, NT, TX, TZ, MIX, HLLC>(a, w - first[lo], S);
    __syncthreads();
  }
}

}  // namespace snap
