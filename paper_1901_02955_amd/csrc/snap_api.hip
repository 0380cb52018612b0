// C-ABI entry points of libsnap: argument validation, workspace layout and
// kernel dispatch. Every argument is checked on the host before the first HIP
// call, so an invalid call never touches the device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/snap.h"
#include "snap_adjoint.h"
#include "snap_internal.h"

using namespace snap;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SNAP_OK;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

bool is3d(const snap_grid* g) { return g->ny > 1; }
int nvar_of(const snap_grid* g) { return 5 + g->ntracer; }
size_t elem_of(const snap_grid* g) { return g->dtype == SNAP_F64 ? 8 : 4; }

long long padded_cells(const snap_grid* g) {
  const long long nyp = is3d(g) ? g->ny + 2 * SNAP_NG : 1;
  return (long long)(g->nx + 2 * SNAP_NG) * nyp * (g->nz + 2 * SNAP_NG);
}

size_t padded_bytes(const snap_grid* g) {
  return (size_t)padded_cells(g) * nvar_of(g) * elem_of(g);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The mixture equation of state is in effect (with no tracers it is the dry gas).
bool uses_mixture(const snap_grid* g) { return g->eos == SNAP_EOS_MIXTURE && g->ntracer > 0; }

// Coefficients of the mixture relation (App. B): a_t = 1/eps_t - 1 for a
// vapour, -1 for a condensate; b_t = sigma_t - 1; mu_t.
Mixture mixture_of(const snap_grid* g) {
  Mixture m;
  memset(&m, 0, sizeof m);
  if (!uses_mixture(g)) return m;
  for (int t = 0; t < g->ntracer; ++t) {
    m.a[t] = g->tracer_kind[t] == SNAP_TRACER_CONDENSATE ? -1.0 : 1.0 / g->tracer_eps[t] - 1.0;
    m.b[t] = g->tracer_sigma[t] - 1.0;
    m.mu[t] = g->tracer_mu[t];
    m.af[t] = (float)m.a[t];
    m.bf[t] = (float)m.b[t];
    m.muf[t] = (float)m.mu[t];
  }
  return m;
}

// Any condensate falls (read only under the mixture).
bool uses_sediment(const snap_grid* g) {
  if (!uses_mixture(g)) return false;
  for (int t = 0; t < g->ntracer; ++t)
    if (g->tracer_wt[t] != 0.0) return true;
  return false;
}

Sediment sediment_of(const snap_grid* g) {
  Sediment d;
  memset(&d, 0, sizeof d);
  if (!uses_sediment(g)) return d;
  d.on = 1;
  d.closed_z = g->bc[2] == SNAP_BC_REFLECT ? 1 : 0;
  d.rd = g->rd;
  d.rdf = (float)g->rd;
  const double cvd = g->rd / (g->gamma - 1.0);
  for (int t = 0; t < g->ntracer; ++t) {
    d.wt[t] = g->tracer_wt[t];
    d.ct[t] = g->tracer_sigma[t] * cvd;
    d.wtf[t] = (float)d.wt[t];
    d.ctf[t] = (float)d.ct[t];
  }
  return d;
}

int check_grid(const snap_grid* g) {
  if (!g) return fail(SNAP_E_INVALID, "grid pointer is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(SNAP_E_INVALID, "grid sizes must be >= 1 (nx=%d ny=%d nz=%d)", g->nx, g->ny, g->nz);
  if (g->nx > (1 << 24) || g->ny > (1 << 24) || g->nz > (1 << 24))
    return fail(SNAP_E_INVALID, "grid size above 2^24 cells along an axis");
  if (g->ng != SNAP_NG) return fail(SNAP_E_INVALID, "ng must be %d (got %d)", SNAP_NG, g->ng);
  if (g->ntracer < 0) return fail(SNAP_E_INVALID, "ntracer must be >= 0 (got %d)", g->ntracer);
  if (g->ntracer > SNAP_MAX_TRACERS)
    return fail(SNAP_E_UNSUPPORTED, "ntracer %d exceeds %d", g->ntracer, SNAP_MAX_TRACERS);
  if (g->dtype != SNAP_F64 && g->dtype != SNAP_F32)
    return fail(SNAP_E_INVALID, "dtype must be SNAP_F64 or SNAP_F32 (got %d)", g->dtype);
  for (int d = 0; d < 3; ++d) {
    if (d == 1 && !is3d(g)) continue;
    if (g->bc[d] != SNAP_BC_PERIODIC && g->bc[d] != SNAP_BC_REFLECT)
      return fail(SNAP_E_INVALID, "bc[%d] must be periodic or reflecting (got %d)", d, g->bc[d]);
  }
  if (g->weno_linear != 0 && g->weno_linear != 1)
    return fail(SNAP_E_INVALID, "weno_linear must be 0 or 1");
  if (!finite_pos(g->dx) || !finite_pos(g->dz) || (is3d(g) && !finite_pos(g->dy)))
    return fail(SNAP_E_INVALID, "cell sizes must be finite and > 0");
  if (!isfinite(g->gamma) || !(g->gamma > 1.0))
    return fail(SNAP_E_INVALID, "gamma must be finite and > 1");
  if (!isfinite(g->grav) || !(g->grav >= 0.0))
    return fail(SNAP_E_INVALID, "grav must be finite and >= 0");
  if (!(g->weno_eps >= 1e-30 && g->weno_eps <= 1e30))
    return fail(SNAP_E_INVALID, "weno_eps must lie in [1e-30, 1e30]");
  if (!g->rhobar_cell || !g->pbar_cell || !g->rhobar_face || !g->pbar_face)
    return fail(SNAP_E_INVALID, "reference profile pointer is NULL");
  if (g->riemann != SNAP_RIEMANN_LMARS && g->riemann != SNAP_RIEMANN_HLLC)
    return fail(SNAP_E_INVALID, "riemann must be SNAP_RIEMANN_LMARS or SNAP_RIEMANN_HLLC (got %d)",
                g->riemann);
  if (g->eos != SNAP_EOS_PASSIVE && g->eos != SNAP_EOS_MIXTURE)
    return fail(SNAP_E_INVALID, "eos must be SNAP_EOS_PASSIVE or SNAP_EOS_MIXTURE (got %d)", g->eos);
  if (g->eos == SNAP_EOS_MIXTURE) {
    for (int t = 0; t < g->ntracer; ++t) {
      const int k = g->tracer_kind[t];
      if (k != SNAP_TRACER_VAPOUR && k != SNAP_TRACER_CONDENSATE)
        return fail(SNAP_E_INVALID, "tracer_kind[%d] must be vapour or condensate (got %d)", t, k);
      if (k == SNAP_TRACER_VAPOUR && !finite_pos(g->tracer_eps[t]))
        return fail(SNAP_E_INVALID, "tracer_eps[%d] must be finite and > 0", t);
      if (!finite_pos(g->tracer_sigma[t]))
        return fail(SNAP_E_INVALID, "tracer_sigma[%d] must be finite and > 0", t);
      if (!isfinite(g->tracer_mu[t]))
        return fail(SNAP_E_INVALID, "tracer_mu[%d] must be finite", t);
      if (!isfinite(g->tracer_wt[t]))
        return fail(SNAP_E_INVALID, "tracer_wt[%d] must be finite", t);
      if (g->tracer_wt[t] != 0.0 && k != SNAP_TRACER_CONDENSATE)
        return fail(SNAP_E_INVALID, "tracer_wt[%d]: only condensates fall", t);
    }
    if (uses_sediment(g) && !finite_pos(g->rd))
      return fail(SNAP_E_INVALID, "rd must be finite and > 0 when a condensate falls");
  }
  if (g->riemann == SNAP_RIEMANN_HLLC && uses_mixture(g))
    return fail(SNAP_E_UNSUPPORTED, "HLLC takes passive tracers (eos = SNAP_EOS_PASSIVE)");
  if (g->storage != SNAP_STORE_TOTAL && g->storage != SNAP_STORE_PERTURBATION)
    return fail(SNAP_E_INVALID, "storage must be SNAP_STORE_TOTAL or SNAP_STORE_PERTURBATION (got %d)",
                g->storage);
  if (g->storage == SNAP_STORE_PERTURBATION && g->eos == SNAP_EOS_MIXTURE)
    return fail(SNAP_E_UNSUPPORTED, "perturbation storage takes passive tracers (eos = SNAP_EOS_PASSIVE)");
  const double total = (double)padded_cells(g) * nvar_of(g);
  if (total > 9.0e18 / 8.0) return fail(SNAP_E_INVALID, "state too large");
  return SNAP_OK;
}

int device_fail(const char* what) {
  const hipError_t e = hipGetLastError();
  return fail(SNAP_E_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

StageArgs stage_args(const snap_grid* g) {
  StageArgs a;
  memset(&a, 0, sizeof a);
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG;
  const long long nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.ry = g->nx;
  a.rz = (long long)g->nx * g->ny;
  a.rv = a.rz * g->nz;
  a.dxi = 1.0 / g->dx;
  a.dyi = d3 ? 1.0 / g->dy : 0.0;
  a.dzi = 1.0 / g->dz;
  a.gamma = g->gamma;
  a.gm1 = g->gamma - 1.0;
  a.inv_gm1 = 1.0 / (g->gamma - 1.0);
  a.grav = g->grav;
  a.eps = g->weno_eps;
  a.linear = g->weno_linear;
  a.rbar_c = g->rhobar_cell;
  a.pbar_c = g->pbar_cell;
  a.rbar_f = g->rhobar_face;
  a.pbar_f = g->pbar_face;
  a.mix = mixture_of(g);
  a.sed = sediment_of(g);
  a.pert = g->storage == SNAP_STORE_PERTURBATION ? 1 : 0;
  a.ghost = (g->bc[0] == SNAP_BC_REFLECT ? GF_RX : 0) |
            (is3d(g) && g->bc[1] == SNAP_BC_REFLECT ? GF_RY : 0) |
            (g->bc[2] == SNAP_BC_REFLECT ? GF_RZ : 0);   // GF_ON is set by the caller
  return a;
}

// Co-resident stage workgroups on the current device (compute units x
// workgroups per compute unit), cached per device, dtype and variable count;
// *cus_out (optional) receives the compute-unit count.
int resident_slots(const snap_grid* g, int* cus_out = nullptr) {
  static std::mutex m;
  static std::vector<std::vector<int>> cache;  // [device][key]
  static std::vector<int> cu_count;            // [device]
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const int kind = (is3d(g) && uses_sediment(g)) ? 3
                   : uses_mixture(g) ? 1 : (g->riemann == SNAP_RIEMANN_HLLC ? 2 : 0);
  const int key = ((g->dtype * 2 + (is3d(g) ? 1 : 0)) * 4 + kind) * 16 + g->ntracer;
  std::lock_guard<std::mutex> lk(m);
  if ((int)cache.size() <= dev) {
    cache.resize(dev + 1);
    cu_count.resize(dev + 1, 0);
  }
  auto& c = cache[dev];
  if (c.empty()) c.assign(256, 0);
  if (c[key] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    const bool d3 = is3d(g);
    int per = kind == 3 ? (g->dtype == SNAP_F64 ? occupancy_sed_f64(g->ntracer)
                                                : occupancy_sed_f32(g->ntracer))
              : g->dtype == SNAP_F64
                  ? (kind == 1 ? occupancy_mix_f64(g->ntracer, d3)
                               : kind == 2 ? occupancy_hllc_f64(g->ntracer, d3) : occupancy_f64(g->ntracer, d3))
                  : (kind == 1 ? occupancy_mix_f32(g->ntracer, d3)
                               : kind == 2 ? occupancy_hllc_f32(g->ntracer, d3) : occupancy_f32(g->ntracer, d3));
    if (per <= 0) per = 1;
    c[key] = cus * per;
    cu_count[dev] = cus;
  }
  if (cus_out) *cus_out = cu_count[dev];
  return c[key];
}

// Relative speed of the workgroups of each dispatch pass when a compute unit
// holds one workgroup of every pass (passes = workgroups per compute unit).
// The wave arbiter favours older waves, so a compute unit's first workgroup
// outpaces the later ones; giving it proportionally more levels lets them
// finish together instead of leaving the last one alone on the compute unit.
// SNAP_STAGE_PASS_WEIGHTS="w0,w1,..." overrides the table (1,1 = even split;
// any value that is not a list of positive numbers, e.g. "off", switches the
// pass mapping off). The compute unit that receives block b of such a launch
// also receives block b + (compute units): the dispatcher fills every compute
// unit once before it places a second workgroup anywhere.
bool pass_weights(const snap_grid* g, int passes, double* w) {
  for (int p = 0; p < passes; ++p) w[p] = 1.0;
  if (const char* env = getenv("SNAP_STAGE_PASS_WEIGHTS")) {
    const char* c = env;
    for (int p = 0; p < passes && *c; ++p) {
      char* end = nullptr;
      const double v = strtod(c, &end);
      if (end == c || !(v > 0.0 && v < 1e30)) return false;   // also rejects inf and nan
      w[p] = v;
      c = *end == ',' ? end + 1 : end;
    }
    return true;
  }
  // measured on the 256 x 256 x 128 convection grid (256 tiles, 256 compute
  // units) with the five conserved variables: 2 passes (double precision)
  // best at 1.5 : 1, stage -8 %; 3 passes (single precision) at
  // 1.35 : 1.35 : 1, stage -10 %. With tracers the kernels' balance differs
  // and the even split is kept.
  if (g->ntracer != 0) return false;
  if (passes == 2) {
    w[0] = 1.5;
    return true;
  }
  if (passes == 3) {
    w[0] = w[1] = 1.35;
    return true;
  }
  return false;
}

// Tiling of the stage launch; returns the number of workgroups.
int stage_tiling(const snap_grid* g, StageArgs& a) {
  const bool d3 = is3d(g);
  const TileShape t = g->dtype == SNAP_F64 ? tile_f64(nvar_of(g)) : tile_f32(nvar_of(g));
  a.tiles_x = (g->nx + t.tx - 1) / t.tx;
  if (!d3) {
    a.tiles_y = (g->nz + t.ty - 1) / t.ty;
    a.nchunk = 1;
    a.tz = g->nz;
    return a.tiles_x * a.tiles_y;
  }
  a.tiles_y = (g->ny + t.ty - 1) / t.ty;
  const int tiles = a.tiles_x * a.tiles_y;
  // Split the levels into chunks. Every chunk pays a warm-up of about one
  // level (two extra vertical reconstructions and primitive loads), and the
  // launch runs in rounds of `slots` co-resident workgroups; pick the chunk
  // count that minimises rounds x (levels per chunk + 1).
  const int slots = resident_slots(g);
  int best = 1;
  double best_cost = 1e300;
  const int maxchunk = g->nz / 4 > 1 ? g->nz / 4 : 1;
  for (int nc = 1; nc <= maxchunk; ++nc) {
    const int tz = (g->nz + nc - 1) / nc;
    const long long blocks = (long long)tiles * ((g->nz + tz - 1) / tz);
    if (blocks > (1LL << 30)) break;
    const long long rounds = (blocks + slots - 1) / slots;
    const double cost = (double)rounds * (tz + 1);
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = nc;
    }
  }
  if (const char* env = getenv("SNAP_STAGE_CHUNKS")) {
    const int nc = atoi(env);
    if (nc >= 1) best = nc < g->nz ? nc : g->nz;
  }
  a.tz = (g->nz + best - 1) / best;
  a.nchunk = (g->nz + a.tz - 1) / a.tz;
  // One workgroup per compute unit per chunk, all resident at once: chunk c is
  // dispatch pass c, and its level range is sized by that pass's speed.
  int cus = 0;
  resident_slots(g, &cus);
  double w[SNAP_MAX_PASSES];
  a.pass_map = 0;
  if (tiles == cus && tiles % 8 == 0 && (long long)tiles * a.nchunk == slots &&
      a.nchunk >= 2 && a.nchunk <= SNAP_MAX_PASSES && pass_weights(g, a.nchunk, w)) {
    double tot = 0.0;
    for (int c = 0; c < a.nchunk; ++c) tot += w[c];
    double acc = 0.0;
    a.kb[0] = 0;
    bool ok = true;
    for (int c = 0; c < a.nchunk; ++c) {
      acc += w[c];
      a.kb[c + 1] = c + 1 == a.nchunk ? g->nz : (int)(g->nz * acc / tot + 0.5);
      if (a.kb[c + 1] - a.kb[c] < 1) ok = false;
    }
    a.pass_map = ok ? 1 : 0;
  }
  return tiles * a.nchunk;
}

// Optional timing of the stage kernels: while enabled, each stage launch is
// bracketed by a pair of hipEvents recorded on the launch stream.
struct StageTiming {
  std::mutex m;
  bool on = false;
  std::vector<hipEvent_t> ev;  // start, stop, start, stop, ...
  size_t used = 0;
};
StageTiming g_timing;

int timing_mark(hipStream_t st) {
  if (g_timing.used == g_timing.ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return device_fail("hipEventCreate");
    g_timing.ev.push_back(e);
  }
  if (hipEventRecord(g_timing.ev[g_timing.used], st) != hipSuccess)
    return device_fail("hipEventRecord");
  ++g_timing.used;
  return SNAP_OK;
}

int run_stage(const snap_grid* g, StageArgs a, hipStream_t st) {
  const int nb = stage_tiling(g, a);
  std::unique_lock<std::mutex> lk(g_timing.m);
  const bool timed = g_timing.on;
  if (!timed) lk.unlock();
  if (timed) {
    const int r = timing_mark(st);
    if (r) return r;
  }
  const bool mix = uses_mixture(g), hllc = g->riemann == SNAP_RIEMANN_HLLC, d3 = is3d(g);
  // 3-D with falling condensates: the sedimentation terms inside the stage kernel
  const bool sed3 = d3 && a.sed.on;
  const int r = sed3 ? (g->dtype == SNAP_F64 ? launch_stage_sed_f64(g->ntracer, a, nb, st)
                                             : launch_stage_sed_f32(g->ntracer, a, nb, st))
                : g->dtype == SNAP_F64
                    ? (mix ? launch_stage_mix_f64(g->ntracer, d3, a, nb, st)
                           : hllc ? launch_stage_hllc_f64(g->ntracer, d3, a, nb, st)
                                  : launch_stage_f64(g->ntracer, d3, a, nb, st))
                    : (mix ? launch_stage_mix_f32(g->ntracer, d3, a, nb, st)
                           : hllc ? launch_stage_hllc_f32(g->ntracer, d3, a, nb, st)
                                  : launch_stage_f32(g->ntracer, d3, a, nb, st));
  if (r != 0) return device_fail("stage kernel launch");
  if (timed) {
    const int t = timing_mark(st);
    if (t) return t;
  }
  // 2-D sedimentation: its part of the right-hand side added to the stage output
  if (a.sed.on && !sed3 && launch_sediment(g->dtype, g->ntracer, a, st))
    return device_fail("sedimentation kernel launch");
  return SNAP_OK;
}

GhostArgs ghost_args(const snap_grid* g);

int fill(const snap_grid* g, void* q, hipStream_t st) {
  const GhostArgs a = ghost_args(g);
  return launch_fill_ghosts(g->dtype, q, a, st) == 0 ? SNAP_OK : device_fail("ghost fill launch");
}

AdjArgs adj_args(const snap_grid* g) {
  AdjArgs a;
  memset(&a, 0, sizeof a);
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG, nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.d3 = d3;
  a.nvar = nvar_of(g);
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.ry = g->nx;
  a.rz = (long long)g->nx * g->ny;
  a.rv = a.rz * g->nz;
  a.dxi[0] = 1.0 / g->dx;
  a.dxi[1] = d3 ? 1.0 / g->dy : 0.0;
  a.dxi[2] = 1.0 / g->dz;
  a.gamma = g->gamma;
  a.gm1 = g->gamma - 1.0;
  a.inv_gm1 = 1.0 / (g->gamma - 1.0);
  a.grav = g->grav;
  a.eps = g->weno_eps;
  a.linear = g->weno_linear;
  for (int d = 0; d < 3; ++d) a.bc[d] = g->bc[d];
  a.pert = g->storage == SNAP_STORE_PERTURBATION ? 1 : 0;
  a.hllc = g->riemann == SNAP_RIEMANN_HLLC ? 1 : 0;
  a.mixture = uses_mixture(g) ? 1 : 0;
  a.mix = mixture_of(g);
  a.sed = sediment_of(g);
  a.rbar_c = g->rhobar_cell;
  a.pbar_c = g->pbar_cell;
  a.rbar_f = g->rhobar_face;
  a.pbar_f = g->pbar_face;
  return a;
}

size_t interior_bytes(const snap_grid* g) {
  return (size_t)g->nx * g->ny * g->nz * nvar_of(g) * elem_of(g);
}

// Layout of the right-hand-side adjoint workspace: P, the padded primitive
// cotangent (the direction kernels convert the state to primitives
// themselves).
struct AdjLayout {
  size_t p, total;
};

AdjLayout adj_layout(const snap_grid* g) {
  AdjLayout L;
  L.p = 0;
  L.total = L.p + align256(padded_bytes(g));
  return L;
}

AdjWork adj_work(const snap_grid* g, void* base) {
  const AdjLayout L = adj_layout(g);
  AdjWork w;
  w.P = static_cast<char*>(base) + L.p;
  return w;
}

// q_bar-like interior array: out = mode 0: J^T rb; 1: out + J^T rb;
// 2: alpha out + beta J^T rb; 3: alpha rb + beta J^T rb; 4: alpha out + gam y
// + rb + beta J^T rb. q must have its ghosts filled.
int run_adj_rhs(const snap_grid* g, void* q, const void* rb, void* out, int mode, double alpha,
                double beta, void* work, hipStream_t st, const void* y = nullptr,
                double gam = 0.0) {
  const AdjArgs a = adj_args(g);
  const AdjWork w = adj_work(g, work);
  const int r = g->dtype == SNAP_F64
                    ? launch_adj_rhs_f64(w, a, q, rb, out, mode, alpha, beta, y, gam, st)
                    : launch_adj_rhs_f32(w, a, q, rb, out, mode, alpha, beta, y, gam, st);
  return r == 0 ? SNAP_OK : device_fail("adjoint kernel launch");
}

// ---------------------------------------------------------------------------
// Ensemble of 2-D domains
// ---------------------------------------------------------------------------
int check_batch(const snap_grid* gs, int n) {
  if (!gs) return fail(SNAP_E_INVALID, "grid array is NULL");
  if (n < 1 || n > 65535) return fail(SNAP_E_INVALID, "member count must lie in [1, 65535]");
  for (int m = 0; m < n; ++m) {
    int r = check_grid(&gs[m]);
    if (r) return fail(r, "member %d: %s", m, g_err.c_str());
    if (is3d(&gs[m]))
      return fail(SNAP_E_UNSUPPORTED, "member %d is 3-D: the batched step takes 2-D members", m);
    if (gs[m].dtype != gs[0].dtype || gs[m].ntracer != gs[0].ntracer)
      return fail(SNAP_E_INVALID, "member %d differs in dtype or ntracer from member 0", m);
    if (uses_mixture(&gs[m]) != uses_mixture(&gs[0]) || gs[m].riemann != gs[0].riemann)
      return fail(SNAP_E_INVALID,
                  "member %d differs from member 0 in its equation of state or Riemann solver", m);
    if (stage_args(&gs[m]).sed.on)
      return fail(SNAP_E_UNSUPPORTED,
                  "member %d has falling condensates: the batched step takes no sedimentation", m);
  }
  return SNAP_OK;
}

struct BatchLayout {
  size_t descs, ghosts, first, members, total;
  std::vector<size_t> q1, q2;
};

BatchLayout batch_layout(const snap_grid* gs, int n) {
  BatchLayout L;
  L.descs = 0;
  L.ghosts = align256((size_t)3 * n * sizeof(StageArgs));
  L.first = L.ghosts + align256((size_t)3 * n * sizeof(GhostDesc));
  L.members = L.first + align256((size_t)(n + 1) * sizeof(int));
  size_t off = L.members;
  L.q1.resize(n);
  L.q2.resize(n);
  for (int m = 0; m < n; ++m) {
    L.q1[m] = off;
    off += align256(padded_bytes(&gs[m]));
    L.q2[m] = off;
    off += align256(padded_bytes(&gs[m]));
  }
  L.total = off;
  return L;
}

GhostArgs ghost_args(const snap_grid* g) {
  GhostArgs a;
  const bool d3 = is3d(g);
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.nxp = g->nx + 2 * SNAP_NG;
  a.nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.gy = d3 ? SNAP_NG : 0;
  a.d3 = d3;
  a.nvar = nvar_of(g);
  a.bcx = g->bc[0];
  a.bcy = g->bc[1];
  a.bcz = g->bc[2];
  a.sy = a.nxp;
  a.sz = (long long)a.nxp * a.nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  return a;
}

}  // namespace

extern "C" {

const char* snap_last_error(void) { return g_err.c_str(); }

int snap_abi_version(void) { return SNAP_ABI_VERSION; }

size_t snap_workspace_bytes(const snap_grid* g, int op) {
  if (check_grid(g) != SNAP_OK) return 0;
  switch (op) {
    case SNAP_OP_RHS: return 0;
    case SNAP_OP_RK3: return 2 * align256(padded_bytes(g));
    case SNAP_OP_RK3_CFL: return 2 * align256(padded_bytes(g)) + 256;
    case SNAP_OP_CFL: return 256;
    case SNAP_OP_SUMS:
      return align256((size_t)SUM_BLOCKS * nvar_of(g) * sizeof(double)) +
             align256(nvar_of(g) * sizeof(double));
    case SNAP_OP_RHS_ADJ: return adj_layout(g).total;
    case SNAP_OP_RK3_ADJ:
      return 2 * align256(padded_bytes(g)) + 2 * align256(interior_bytes(g)) +
             adj_layout(g).total;
    default: fail(SNAP_E_INVALID, "unknown workspace operation %d", op); return 0;
  }
}

int snap_stage_timing_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_timing.m);
  g_timing.on = enable != 0;
  g_timing.used = 0;
  return ok();
}

int snap_stage_timing_read(double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return fail(SNAP_E_INVALID, "total_ms or launches is NULL");
  std::lock_guard<std::mutex> lk(g_timing.m);
  double sum = 0.0;
  for (size_t i = 0; i + 1 < g_timing.used; i += 2) {
    if (hipEventSynchronize(g_timing.ev[i + 1]) != hipSuccess)
      return device_fail("hipEventSynchronize");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, g_timing.ev[i], g_timing.ev[i + 1]) != hipSuccess)
      return device_fail("hipEventElapsedTime");
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)(g_timing.used / 2);
  return ok();
}

int snap_fill_ghosts(const snap_grid* g, void* q, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q) return fail(SNAP_E_INVALID, "q is NULL");
  r = fill(g, q, (hipStream_t)stream);
  return r ? r : ok();
}

int snap_rhs(const snap_grid* g, void* q, void* rhs, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !rhs) return fail(SNAP_E_INVALID, "q or rhs is NULL");
  if (q == rhs) return fail(SNAP_E_INVALID, "rhs must not alias q");
  const hipStream_t st = (hipStream_t)stream;
  if ((r = fill(g, q, st))) return r;
  StageArgs a = stage_args(g);
  a.qs = q;
  a.qn = nullptr;
  a.out = rhs;
  a.rhs_mode = 1;
  if ((r = run_stage(g, a, st))) return r;
  return ok();
}

}  // extern "C"

namespace {

// Arguments of the maximum-signal-speed reduction (snap_cfl_dt).
CflArgs cfl_args(const snap_grid* g) {
  CflArgs a;
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG, nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.d3 = d3;
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.gamma = g->gamma;
  a.gm1 = g->gamma - 1.0;
  a.dxi = 1.0 / g->dx;
  a.dyi = 1.0 / g->dy;
  a.dzi = 1.0 / g->dz;
  a.ntracer = g->ntracer;
  a.mix = uses_mixture(g) ? 1 : 0;
  a.m = mixture_of(g);
  a.pert = g->storage == SNAP_STORE_PERTURBATION ? 1 : 0;
  a.rbar_c = g->rhobar_cell;
  a.pbar_c = g->pbar_cell;
  return a;
}

// The three stages of one SSP-RK3 step (Sec. 4.3) on validated arguments.
// dt is taken from the host (smax == nullptr) or, on the device, as
// cfl / *smax; dt_out (device, optional) receives the dt of the first stage.
// smax_next (only where fused_speed_ok): the first stage clears it and the
// last reduces the new state's maximum signal speed into it.
int rk3_stages(const snap_grid* g, void* q, double dt, const unsigned long long* smax,
               double cfl, double* dt_out, char* w, hipStream_t st,
               unsigned long long* smax_next = nullptr,
               unsigned long long* state_flag = nullptr) {
  int r;
  void* q1 = w;
  void* q2 = w + align256(padded_bytes(g));
  StageArgs a = stage_args(g);
  a.dt = dt;
  a.smax = smax;
  a.cfl = cfl;
  a.rhs_mode = 0;
  // The 3-D stage kernels without tracers read the ghost cells they need at
  // their sources, so their input needs no fill; the sedimentation kernel
  // still reads z ghosts.
  if (is3d(g) && !a.sed.on && ghosts_in_place(g->ntracer)) a.ghost |= GF_ON;
  auto prepare = [&](void* x) { return (a.ghost & GF_ON) ? SNAP_OK : fill(g, x, st); };
  // Q1 = Q + dt R(Q)
  if ((r = prepare(q))) return r;
  a.qs = q;
  a.qn = nullptr;
  a.out = q1;
  a.ca = 0.0;
  a.cb = 1.0;
  a.dt_out = dt_out;
  a.smax_zero = smax_next;
  a.state_flag = state_flag;
  if ((r = run_stage(g, a, st))) return r;
  a.dt_out = nullptr;
  a.smax_zero = nullptr;
  a.state_flag = nullptr;
  // Q2 = 3/4 Q + 1/4 (Q1 + dt R(Q1))
  if ((r = prepare(q1))) return r;
  a.qs = q1;
  a.qn = q;
  a.out = q2;
  a.ca = 0.75;
  a.cb = 0.25;
  if ((r = run_stage(g, a, st))) return r;
  // Q <- 1/3 Q + 2/3 (Q2 + dt R(Q2)), in place (each cell reads only its own Q)
  if ((r = prepare(q2))) return r;
  a.qs = q2;
  a.qn = q;
  a.out = q;
  a.ca = 1.0 / 3.0;
  a.cb = 2.0 / 3.0;
  a.smax_out = smax_next;
  if ((r = run_stage(g, a, st))) return r;
  return ok();
}

// Grids whose last stage can reduce the next step's signal speed itself
// (fused_speed in the kernels: no tracers, 3-D, ghosts read in place, i.e. no
// sedimentation).
bool fused_speed_ok(const snap_grid* g) {
  return is3d(g) && ghosts_in_place(g->ntracer) && !sediment_of(g).on;
}

// The 256 bytes after the two padded stage states of the SNAP_OP_RK3_CFL
// workspace: two signal-speed slots, then the state flag.
unsigned long long* cfl_slots(const snap_grid* g, void* work) {
  return reinterpret_cast<unsigned long long*>(static_cast<char*>(work) +
                                               2 * align256(padded_bytes(g)));
}

// nsteps SSP-RK3 steps with the time step formed on the device. The maximum
// signal speed of Q^n lives in one of two slots after the RK3 workspace: the
// first comes from the reduction kernel; each later one from the previous
// step's last stage where the kernels can fuse it, else from the kernel.
// The state flag (the third word) is cleared first; the first stage of every
// step raises it when its time step is not finite and positive, and where the
// kernels fuse the reduction the last step also reduces the final state, which
// a one-thread kernel then checks.
int rk3_steps_cfl(const snap_grid* g, void* q, double cfl, int nsteps, void* work,
                  double* dt_dev, hipStream_t st) {
  char* w = static_cast<char*>(work);
  unsigned long long* slot = cfl_slots(g, work);
  unsigned long long* flag = slot + 2;
  const bool fused = fused_speed_ok(g);
  const CflArgs ca = cfl_args(g);
  if (launch_zero_u64(flag, 1, st)) return device_fail("flag clear launch");
  if (launch_cfl(g->dtype, q, ca, slot, st)) return device_fail("cfl kernel launch");
  for (int n = 0; n < nsteps; ++n) {
    unsigned long long* cur = slot + (n & 1);
    unsigned long long* nxt = slot + ((n + 1) & 1);
    const bool more = n + 1 < nsteps;
    const int r = rk3_stages(g, q, 0.0, cur, cfl, dt_dev ? dt_dev + n : nullptr, w, st,
                             fused ? nxt : nullptr, flag);
    if (r) return r;
    if (more && !fused && launch_cfl(g->dtype, q, ca, nxt, st))
      return device_fail("cfl kernel launch");
  }
  if (fused && launch_flag_speed(slot + (nsteps & 1), flag, st))
    return device_fail("flag kernel launch");
  return ok();
}


}  // namespace

extern "C" {

int snap_rk3_step(const snap_grid* g, void* q, double dt, void* work, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q) return fail(SNAP_E_INVALID, "q is NULL");
  if (!work) return fail(SNAP_E_INVALID, "work is NULL");
  if (!finite_pos(dt)) return fail(SNAP_E_INVALID, "dt must be finite and > 0");
  return rk3_stages(g, q, dt, nullptr, 0.0, nullptr, static_cast<char*>(work),
                    (hipStream_t)stream);
}

int snap_rk3_step_cfl(const snap_grid* g, void* q, double cfl, void* work, double* dt_dev,
                      void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q) return fail(SNAP_E_INVALID, "q is NULL");
  if (!work) return fail(SNAP_E_INVALID, "work is NULL");
  if (!finite_pos(cfl)) return fail(SNAP_E_INVALID, "cfl must be finite and > 0");
  return rk3_steps_cfl(g, q, cfl, 1, work, dt_dev, (hipStream_t)stream);
}

int snap_rk3_steps_cfl(const snap_grid* g, void* q, double cfl, int nsteps, void* work,
                       double* dt_dev, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q) return fail(SNAP_E_INVALID, "q is NULL");
  if (!work) return fail(SNAP_E_INVALID, "work is NULL");
  if (!finite_pos(cfl)) return fail(SNAP_E_INVALID, "cfl must be finite and > 0");
  if (nsteps < 1) return fail(SNAP_E_INVALID, "nsteps must be >= 1");
  return rk3_steps_cfl(g, q, cfl, nsteps, work, dt_dev, (hipStream_t)stream);
}

int snap_rk3_steps_status(const snap_grid* g, void* work, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!work) return fail(SNAP_E_INVALID, "work is NULL");
  const hipStream_t st = (hipStream_t)stream;
  unsigned long long flag = 0;
  if (hipMemcpyAsync(&flag, cfl_slots(g, work) + 2, sizeof flag, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return device_fail("state flag copy");
  if (hipStreamSynchronize(st) != hipSuccess) return device_fail("state flag synchronize");
  if (flag != 0)
    return fail(SNAP_E_STATE,
                "a step of the last device-dt call met a non-finite or non-positive density or "
                "pressure (its time step and every later state are not finite)");
  return ok();
}

int snap_rhs_adjoint(const snap_grid* g, void* q, const void* rhs_bar, void* q_bar, void* work,
                     void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !rhs_bar || !q_bar || !work)
    return fail(SNAP_E_INVALID, "q, rhs_bar, q_bar or work is NULL");
  if (q_bar == q || q_bar == rhs_bar) return fail(SNAP_E_INVALID, "q_bar must not alias q or rhs_bar");
  const hipStream_t st = (hipStream_t)stream;
  if ((r = fill(g, q, st))) return r;
  if ((r = run_adj_rhs(g, q, rhs_bar, q_bar, 0, 0.0, 1.0, work, st))) return r;
  return ok();
}

// Checks shared by both RK3 adjoint entry points.
static int check_rk3_adjoint(const snap_grid* g, const void* q_n, double dt, const void* q_bar,
                             const void* work) {
  int r = check_grid(g);
  if (r) return r;
  if (!q_n || !q_bar || !work) return fail(SNAP_E_INVALID, "q_n, q_bar or work is NULL");
  if (!finite_pos(dt)) return fail(SNAP_E_INVALID, "dt must be finite and > 0");
  return SNAP_OK;
}

// Reverse of the three stages, given Q, Q1 and Q2 with their ghost cells
// filled (no kernel below writes them); b2, b1: interior scratch; aw: the
// right-hand-side adjoint's workspace.
static int rk3_adjoint_reverse(const snap_grid* g, void* q_n, void* q1, void* q2, double dt,
                               void* q_bar, void* b2, void* b1, void* aw, hipStream_t st) {
  int r;
  // Q3 = Q/3 + 2/3 (Q2 + dt R(Q2)):  B2 = 2/3 (Qb3 + dt J(Q2)^T Qb3)
  if ((r = run_adj_rhs(g, q2, q_bar, b2, 3, 2.0 / 3.0, 2.0 / 3.0 * dt, aw, st))) return r;
  // Q2 = 3/4 Q + 1/4 (Q1 + dt R(Q1)):  B1 = 1/4 (B2 + dt J(Q1)^T B2)
  if ((r = run_adj_rhs(g, q1, b2, b1, 3, 0.25, 0.25 * dt, aw, st))) return r;
  // Q1 = Q + dt R(Q):  Qb = Qb3/3 + 3/4 B2 + B1 + dt J(Q)^T B1 (one pass)
  return run_adj_rhs(g, q_n, b1, q_bar, 4, 1.0 / 3.0, dt, aw, st, b2, 0.75);
}

int snap_rk3_step_adjoint(const snap_grid* g, void* q_n, double dt, void* q_bar, void* work,
                          void* stream) {
  int r = check_rk3_adjoint(g, q_n, dt, q_bar, work);
  if (r) return r;
  const hipStream_t st = (hipStream_t)stream;
  char* b = static_cast<char*>(work);
  void* q1 = b;
  void* q2 = b + align256(padded_bytes(g));
  void* b2 = b + 2 * align256(padded_bytes(g));
  void* b1 = static_cast<char*>(b2) + align256(interior_bytes(g));
  void* aw = static_cast<char*>(b1) + align256(interior_bytes(g));
  // recompute the stage states Q1 and Q2 of the forward step
  StageArgs a = stage_args(g);
  a.dt = dt;
  a.rhs_mode = 0;
  if ((r = fill(g, q_n, st))) return r;
  a.qs = q_n;
  a.qn = nullptr;
  a.out = q1;
  a.ca = 0.0;
  a.cb = 1.0;
  if ((r = run_stage(g, a, st))) return r;
  if ((r = fill(g, q1, st))) return r;
  a.qs = q1;
  a.qn = q_n;
  a.out = q2;
  a.ca = 0.75;
  a.cb = 0.25;
  if ((r = run_stage(g, a, st))) return r;
  if ((r = fill(g, q2, st))) return r;
  if ((r = rk3_adjoint_reverse(g, q_n, q1, q2, dt, q_bar, b2, b1, aw, st))) return r;
  return ok();
}

int snap_rk3_step_adjoint_stages(const snap_grid* g, void* q_n, void* stages, double dt,
                                 void* q_bar, void* work, void* stream) {
  int r = check_rk3_adjoint(g, q_n, dt, q_bar, work);
  if (r) return r;
  if (!stages) return fail(SNAP_E_INVALID, "stages is NULL");
  const hipStream_t st = (hipStream_t)stream;
  // the stage states as snap_rk3_step leaves them in its workspace
  void* q1 = stages;
  void* q2 = static_cast<char*>(stages) + align256(padded_bytes(g));
  char* b = static_cast<char*>(work);
  void* b2 = b + 2 * align256(padded_bytes(g));
  void* b1 = static_cast<char*>(b2) + align256(interior_bytes(g));
  void* aw = static_cast<char*>(b1) + align256(interior_bytes(g));
  if ((r = fill(g, q_n, st))) return r;
  if ((r = fill(g, q1, st))) return r;
  if ((r = fill(g, q2, st))) return r;
  if ((r = rk3_adjoint_reverse(g, q_n, q1, q2, dt, q_bar, b2, b1, aw, st))) return r;
  return ok();
}

size_t snap_batched_workspace_bytes(const snap_grid* gs, int n) {
  if (check_batch(gs, n) != SNAP_OK) return 0;
  return batch_layout(gs, n).total;
}

int snap_batched_tile_variant(int dtype, int ntracer, int variant, int* tx, int* tz) {
  if (!tx || !tz) return fail(SNAP_E_INVALID, "tx or tz is NULL");
  if (dtype != SNAP_F64 && dtype != SNAP_F32) return fail(SNAP_E_INVALID, "bad dtype");
  if (ntracer < 0 || ntracer > SNAP_MAX_TRACERS) return fail(SNAP_E_INVALID, "bad ntracer");
  const TileShape t = batched_tile(dtype, ntracer, variant);
  if (t.tx == 0) return fail(SNAP_E_UNSUPPORTED, "tile variant %d unavailable", variant);
  *tx = t.tx;
  *tz = t.ty;
  return ok();
}

int snap_rk3_step_batched(const snap_grid* gs, int n, void* const* q, const double* dt_host,
                          int variant, int nblocks, void* work, void* stream) {
  int r = check_batch(gs, n);
  if (r) return r;
  if (!q || !dt_host || !work) return fail(SNAP_E_INVALID, "q, dt_host or work is NULL");
  for (int m = 0; m < n; ++m) {
    if (!q[m]) return fail(SNAP_E_INVALID, "q[%d] is NULL", m);
    if (!finite_pos(dt_host[m])) return fail(SNAP_E_INVALID, "dt[%d] must be finite and > 0", m);
  }
  if (nblocks < 0) return fail(SNAP_E_INVALID, "nblocks must be >= 0");
  const int dtype = gs[0].dtype, nt = gs[0].ntracer;
  const int form = uses_mixture(&gs[0]) ? 1 : (gs[0].riemann == SNAP_RIEMANN_HLLC ? 2 : 0);
  const TileShape t = batched_tile(dtype, nt, variant);
  if (t.tx == 0) return fail(SNAP_E_UNSUPPORTED, "tile variant %d unavailable", variant);
  const hipStream_t st = (hipStream_t)stream;
  const BatchLayout L = batch_layout(gs, n);
  char* base = static_cast<char*>(work);

  // host-side descriptor tables: 3 stages x n members, then the item offsets
  thread_local std::vector<char> host;
  host.assign(L.members, 0);
  StageArgs* hd = reinterpret_cast<StageArgs*>(host.data() + L.descs);
  GhostDesc* hg = reinterpret_cast<GhostDesc*>(host.data() + L.ghosts);
  int* hf = reinterpret_cast<int*>(host.data() + L.first);
  long long items = 0, max_ghosts = 0;
  for (int m = 0; m < n; ++m) {
    const snap_grid* g = &gs[m];
    StageArgs a = stage_args(g);
    a.tiles_x = (g->nx + t.tx - 1) / t.tx;
    a.tiles_y = (g->nz + t.ty - 1) / t.ty;
    a.nchunk = 1;
    a.tz = g->nz;
    a.dt = dt_host[m];
    a.rhs_mode = 0;
    void* q1 = base + L.q1[m];
    void* q2 = base + L.q2[m];
    StageArgs s1 = a, s2 = a, s3 = a;
    s1.qs = q[m], s1.qn = nullptr, s1.out = q1, s1.ca = 0.0, s1.cb = 1.0;
    s2.qs = q1, s2.qn = q[m], s2.out = q2, s2.ca = 0.75, s2.cb = 0.25;
    s3.qs = q2, s3.qn = q[m], s3.out = q[m], s3.ca = 1.0 / 3.0, s3.cb = 2.0 / 3.0;
    hd[m] = s1;
    hd[n + m] = s2;
    hd[2 * n + m] = s3;
    const GhostArgs ga = ghost_args(g);
    hg[m] = GhostDesc{ga, q[m]};
    hg[n + m] = GhostDesc{ga, q1};
    hg[2 * n + m] = GhostDesc{ga, q2};
    hf[m] = (int)items;
    items += (long long)a.tiles_x * a.tiles_y;
    const long long ng = 6LL * ga.nyp * ga.nxp + (long long)ga.nz * ga.ny * 6;
    max_ghosts = ng > max_ghosts ? ng : max_ghosts;
  }
  if (items > (1LL << 30)) return fail(SNAP_E_INVALID, "too many tiles in the batch");
  hf[n] = (int)items;
  if (hipMemcpyAsync(base, host.data(), L.members, hipMemcpyHostToDevice, st) != hipSuccess)
    return device_fail("descriptor copy");
  int nb = nblocks;
  if (nb == 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    int per = batched_occupancy(dtype, nt, variant, form);
    nb = cus * (per > 0 ? per : 1);
  }
  if (nb > items) nb = (int)items;
  const StageArgs* dd = reinterpret_cast<const StageArgs*>(base + L.descs);
  const GhostDesc* dg = reinterpret_cast<const GhostDesc*>(base + L.ghosts);
  const int* df = reinterpret_cast<const int*>(base + L.first);
  for (int s = 0; s < 3; ++s) {
    if (launch_fill_ghosts_batched(dtype, dg + s * n, n, max_ghosts, st))
      return device_fail("batched ghost fill launch");
    if (launch_stage2d_batched(dtype, nt, variant, form, dd + s * n, df, n, nb, st))
      return device_fail("batched stage launch");
  }
  return ok();
}

// Validated kernel arguments of a Kessler step (forward or adjoint).
static int kessler_args(const snap_grid* g, double dt, const snap_kessler* k, KesslerArgs& a) {
  if (!finite_pos(dt)) return fail(SNAP_E_INVALID, "dt must be finite and > 0");
  if (!uses_mixture(g))
    return fail(SNAP_E_INVALID, "the microphysics needs eos = SNAP_EOS_MIXTURE and tracers");
  if (k->nspecies < 1 || k->nspecies > SNAP_KESSLER_MAX_SPECIES)
    return fail(SNAP_E_INVALID, "nspecies must lie in [1, %d]", SNAP_KESSLER_MAX_SPECIES);
  if (!finite_pos(k->rd)) return fail(SNAP_E_INVALID, "rd must be finite and > 0");
  if (k->max_iter < 1 || k->max_iter > 100) return fail(SNAP_E_INVALID, "max_iter must lie in [1, 100]");
  if (!isfinite(k->tol) || k->tol < 0.0) return fail(SNAP_E_INVALID, "tol must be finite and >= 0");
  memset(&a, 0, sizeof a);
  bool used[SNAP_MAX_TRACERS] = {false};
  for (int sidx = 0; sidx < k->nspecies; ++sidx) {
    const snap_kessler_species& sp = k->species[sidx];
    const int idx[3] = {sp.vapour, sp.cloud, sp.precip};
    for (int m = 0; m < 3; ++m) {
      if (idx[m] < 0 || idx[m] >= g->ntracer)
        return fail(SNAP_E_INVALID, "species %d: tracer index %d outside [0, %d)", sidx, idx[m], g->ntracer);
      if (used[idx[m]]) return fail(SNAP_E_INVALID, "species %d: tracer %d used twice", sidx, idx[m]);
      used[idx[m]] = true;
      const int want = m == 0 ? SNAP_TRACER_VAPOUR : SNAP_TRACER_CONDENSATE;
      if (g->tracer_kind[idx[m]] != want)
        return fail(SNAP_E_INVALID, "species %d: tracer %d must be a %s", sidx, idx[m],
                    m == 0 ? "vapour" : "condensate");
    }
    const double kk[4] = {sp.k1, sp.k2, sp.k3, sp.k4};
    for (int m = 0; m < 4; ++m)
      if (!isfinite(kk[m]) || kk[m] < 0.0)
        return fail(SNAP_E_INVALID, "species %d: k%d must be finite and >= 0", sidx, m + 1);
    if (!finite_pos(sp.p_ref) || !finite_pos(sp.t_ref))
      return fail(SNAP_E_INVALID, "species %d: p_ref and t_ref must be finite and > 0", sidx);
    if (!isfinite(sp.beta) || !isfinite(sp.delta))
      return fail(SNAP_E_INVALID, "species %d: beta and delta must be finite", sidx);
    KesslerSpec& d = a.s[sidx];
    d.v = sp.vapour;
    d.c = sp.cloud;
    d.p = sp.precip;
    d.k1 = sp.k1;
    d.k2 = sp.k2;
    d.k3 = sp.k3;
    d.k4 = sp.k4;
    d.p_ref = sp.p_ref;
    d.t_ref = sp.t_ref;
    d.beta = sp.beta;
    d.delta = sp.delta;
    d.eps = g->tracer_eps[sp.vapour];
  }
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG, nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.nspecies = k->nspecies;
  a.max_iter = k->max_iter;
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.dt = dt;
  a.rd = k->rd;
  a.tol = k->tol;
  a.gm1 = g->gamma - 1.0;
  a.m = mixture_of(g);
  for (int t = 0; t < g->ntracer; ++t) {
    a.vap[t] = g->tracer_kind[t] == SNAP_TRACER_VAPOUR ? 1 : 0;
    a.eps[t] = a.vap[t] ? g->tracer_eps[t] : 1.0;
  }
  if ((long long)g->ny * g->nz > 0x7fffffffLL) return fail(SNAP_E_INVALID, "ny nz too large");
  return 0;
}

int snap_kessler_step(const snap_grid* g, void* q, double dt, const snap_kessler* k,
                      void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !k) return fail(SNAP_E_INVALID, "q or k is NULL");
  KesslerArgs a;
  if ((r = kessler_args(g, dt, k, a))) return r;
  if (launch_kessler(g->dtype, g->ntracer, q, a, (hipStream_t)stream))
    return device_fail("microphysics kernel launch");
  return ok();
}

int snap_kessler_step_adjoint(const snap_grid* g, const void* q, double dt, const snap_kessler* k,
                              void* q_bar, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !k || !q_bar) return fail(SNAP_E_INVALID, "q, k or q_bar is NULL");
  if (q_bar == q) return fail(SNAP_E_INVALID, "q_bar must not alias q");
  KesslerArgs a;
  if ((r = kessler_args(g, dt, k, a))) return r;
  if (launch_kessler_adj(g->dtype, g->ntracer, q, q_bar, a, (hipStream_t)stream))
    return device_fail("microphysics adjoint kernel launch");
  return ok();
}

static int satadj_args(const snap_grid* g, const snap_satadj* sa, SatAdjArgs& a) {
  if (!uses_mixture(g))
    return fail(SNAP_E_INVALID, "the adjustment needs eos = SNAP_EOS_MIXTURE and tracers");
  if (sa->nspecies < 1 || sa->nspecies > SNAP_SATADJ_MAX_SPECIES)
    return fail(SNAP_E_INVALID, "nspecies must lie in [1, %d]", SNAP_SATADJ_MAX_SPECIES);
  if (!finite_pos(sa->rd)) return fail(SNAP_E_INVALID, "rd must be finite and > 0");
  if (sa->max_iter < 1 || sa->max_iter > 100) return fail(SNAP_E_INVALID, "max_iter must lie in [1, 100]");
  if (!isfinite(sa->tol) || sa->tol < 0.0) return fail(SNAP_E_INVALID, "tol must be finite and >= 0");
  memset(&a, 0, sizeof a);
  bool used[SNAP_MAX_TRACERS] = {false};
  for (int sidx = 0; sidx < sa->nspecies; ++sidx) {
    const snap_satadj_species& sp = sa->species[sidx];
    const int idx[2] = {sp.vapour, sp.cloud};
    for (int m = 0; m < 2; ++m) {
      if (idx[m] < 0 || idx[m] >= g->ntracer)
        return fail(SNAP_E_INVALID, "species %d: tracer index %d outside [0, %d)", sidx, idx[m], g->ntracer);
      if (used[idx[m]]) return fail(SNAP_E_INVALID, "species %d: tracer %d used twice", sidx, idx[m]);
      used[idx[m]] = true;
      const int want = m == 0 ? SNAP_TRACER_VAPOUR : SNAP_TRACER_CONDENSATE;
      if (g->tracer_kind[idx[m]] != want)
        return fail(SNAP_E_INVALID, "species %d: tracer %d must be a %s", sidx, idx[m],
                    m == 0 ? "vapour" : "condensate");
    }
    if (!finite_pos(sp.p_ref) || !finite_pos(sp.t_ref))
      return fail(SNAP_E_INVALID, "species %d: p_ref and t_ref must be finite and > 0", sidx);
    if (!isfinite(sp.beta) || !isfinite(sp.delta))
      return fail(SNAP_E_INVALID, "species %d: beta and delta must be finite", sidx);
    SatAdjSpec& d = a.s[sidx];
    d.v = sp.vapour;
    d.c = sp.cloud;
    d.p_ref = sp.p_ref;
    d.t_ref = sp.t_ref;
    d.beta = sp.beta;
    d.delta = sp.delta;
    d.rv = sa->rd / g->tracer_eps[sp.vapour];
  }
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG, nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.nspecies = sa->nspecies;
  a.max_iter = sa->max_iter;
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.tol = sa->tol;
  a.cvd = sa->rd / (g->gamma - 1.0);
  for (int t = 0; t < g->ntracer; ++t) {
    a.sigma[t] = g->tracer_sigma[t];
    a.mu[t] = g->tracer_mu[t];
  }
  if ((long long)g->ny * g->nz > 0x7fffffffLL) return fail(SNAP_E_INVALID, "ny nz too large");
  return 0;
}

int snap_saturation_adjust(const snap_grid* g, void* q, const snap_satadj* sa, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !sa) return fail(SNAP_E_INVALID, "q or s is NULL");
  SatAdjArgs a;
  if ((r = satadj_args(g, sa, a))) return r;
  if (launch_satadj(g->dtype, g->ntracer, q, a, (hipStream_t)stream))
    return device_fail("saturation adjustment kernel launch");
  return ok();
}

int snap_saturation_adjust_adjoint(const snap_grid* g, const void* q, const snap_satadj* sa,
                                   void* q_bar, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !sa || !q_bar) return fail(SNAP_E_INVALID, "q, s or q_bar is NULL");
  if (q_bar == q) return fail(SNAP_E_INVALID, "q_bar must not alias q");
  SatAdjArgs a;
  if ((r = satadj_args(g, sa, a))) return r;
  if (launch_satadj_adj(g->dtype, g->ntracer, q, q_bar, a, (hipStream_t)stream))
    return device_fail("saturation adjustment adjoint kernel launch");
  return ok();
}

int snap_cfl_dt(const snap_grid* g, void* q, double cfl, void* work, double* dt_host,
                void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !work || !dt_host) return fail(SNAP_E_INVALID, "q, work or dt_host is NULL");
  if (!finite_pos(cfl)) return fail(SNAP_E_INVALID, "cfl must be finite and > 0");
  const hipStream_t st = (hipStream_t)stream;
  const CflArgs a = cfl_args(g);
  unsigned long long* dmax = static_cast<unsigned long long*>(work);
  if (launch_cfl(g->dtype, q, a, dmax, st)) return device_fail("cfl kernel launch");
  unsigned long long bits = 0;
  if (hipMemcpyAsync(&bits, dmax, sizeof bits, hipMemcpyDeviceToHost, st) != hipSuccess)
    return device_fail("cfl copy");
  if (hipStreamSynchronize(st) != hipSuccess) return device_fail("cfl synchronize");
  double smax;
  memcpy(&smax, &bits, sizeof smax);
  if (bits >= 0x7FF0000000000000ULL || !(smax > 0.0))
    return fail(SNAP_E_STATE, "non-finite or non-positive density or pressure in the state");
  *dt_host = cfl / smax;
  return ok();
}

}  // extern "C"

namespace {

// Conservation sums on validated arguments: partials in part[SUM_BLOCKS][nvar]
// and the nvar results in out (device), copied to sums_host.
int run_sums(const snap_grid* g, void* q, double* part, double* out, double* sums_host,
             hipStream_t st) {
  SumArgs a;
  const bool d3 = is3d(g);
  const long long nxp = g->nx + 2 * SNAP_NG, nyp = d3 ? g->ny + 2 * SNAP_NG : 1;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.gy = d3 ? SNAP_NG : 0;
  a.nvar = nvar_of(g);
  a.sy = nxp;
  a.sz = nxp * nyp;
  a.sv = a.sz * (g->nz + 2 * SNAP_NG);
  a.pert = g->storage == SNAP_STORE_PERTURBATION ? 1 : 0;
  a.inv_gm1 = 1.0 / (g->gamma - 1.0);
  a.rbar_c = g->rhobar_cell;
  a.pbar_c = g->pbar_cell;
  if (launch_sums(g->dtype, q, a, part, out, st)) return device_fail("sums kernel launch");
  if (hipMemcpyAsync(sums_host, out, a.nvar * sizeof(double), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return device_fail("sums copy");
  if (hipStreamSynchronize(st) != hipSuccess) return device_fail("sums synchronize");
  return ok();
}

// Offset (doubles) of the results after the partials of nvar variables.
size_t sums_out_offset(int nvar) {
  return align256((size_t)SUM_BLOCKS * nvar * sizeof(double)) / sizeof(double);
}

// Library-owned scratch of snap_conservation_sums_noalloc: the partials of up
// to 5 + SNAP_MAX_TRACERS variables, then the results. Each GPU holds its own
// copy at its own address; host code uses that address (from
// hipGetSymbolAddress), never the array's name, which on the host is only a
// stand-in.
constexpr size_t NOALLOC_SUM_DOUBLES = SNAP_SUMS_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert((size_t)SUM_BLOCKS * (5 + SNAP_MAX_TRACERS) + 5 + SNAP_MAX_TRACERS <=
                  NOALLOC_SUM_DOUBLES,
              "the sums scratch holds every valid grid's partials");
static __device__ __align__(256) double scratch[NOALLOC_SUM_DOUBLES];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch;   // per device ordinal: device address of its scratch

// Device address of the current device's scratch, looked up once per device
// (with that device current) on its first use.
int sums_scratch(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return device_fail("hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(SNAP_E_DEVICE, "hipGetSymbolAddress of the sums scratch failed on device %d: %s",
                  dev, hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return SNAP_OK;
}

}  // namespace

extern "C" {

int snap_conservation_sums(const snap_grid* g, void* q, void* work, double* sums_host,
                           void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !work || !sums_host) return fail(SNAP_E_INVALID, "q, work or sums_host is NULL");
  double* part = static_cast<double*>(work);
  return run_sums(g, q, part, part + sums_out_offset(nvar_of(g)), sums_host, (hipStream_t)stream);
}

int snap_conservation_sums_noalloc(const snap_grid* g, void* q, double* sums_host, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!q || !sums_host) return fail(SNAP_E_INVALID, "q or sums_host is NULL");
  const int nv = nvar_of(g);
  if (sums_out_offset(nv) + nv > NOALLOC_SUM_DOUBLES)
    return fail(SNAP_E_INVALID, "%d variables need %zu bytes of sums scratch, more than the %zu held",
                nv, (sums_out_offset(nv) + nv) * sizeof(double), NOALLOC_SUM_DOUBLES * sizeof(double));
  double* part = nullptr;
  if ((r = sums_scratch(&part))) return r;
  return run_sums(g, q, part, part + sums_out_offset(nv), sums_host, (hipStream_t)stream);
}

}  // extern "C"
