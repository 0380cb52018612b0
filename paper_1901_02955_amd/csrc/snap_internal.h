// Internal declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "snap_stage.h"

namespace snap {

constexpr int CFL_BLOCKS = 2048;
constexpr int SUM_BLOCKS = 512;

struct GhostArgs {
  int nx, ny, nz, nxp, nyp, gy, d3, nvar;
  int bcx, bcy, bcz;
  long long sy, sz, sv;
};

// Ghost fill of one ensemble member.
struct GhostDesc {
  GhostArgs a;
  void* q;
};

struct CflArgs {
  int nx, ny, nz, gy, d3;
  long long sy, sz, sv;
  double gamma, gm1, dxi, dyi, dzi;   // dxi = 1 / dx (x, y, z)
  int ntracer, mix;   // mix: the mixture equation of state with coefficients m
  Mixture m;
  int pert;                       // perturbation storage: add the level references back
  const double* rbar_c;           // nz + 6 (read only with pert)
  const double* pbar_c;
};

// Kessler microphysics (Sec. 3): one condensable species.
struct KesslerSpec {
  int v, c, p;   // tracer indices of vapour, cloud, precipitation
  double k1, k2, k3, k4, p_ref, t_ref, beta, delta, eps;
};

struct KesslerArgs {
  int nx, ny, nz, gy, nspecies, max_iter;
  long long sy, sz, sv;
  double dt, rd, tol, gm1;
  Mixture m;                      // mixture coefficients of the pressure
  int vap[MAX_TRACERS];           // 1: tracer t is a vapour
  double eps[MAX_TRACERS];        // molar-mass ratios of the tracers
  KesslerSpec s[MAX_TRACERS / 3];
};

struct SatAdjSpec {
  int v, c;                            // tracer indices of vapour and cloud
  double p_ref, t_ref, beta, delta, rv;   // rv = R_d / eps of the vapour
};

struct SatAdjArgs {
  int nx, ny, nz, gy, nspecies, max_iter;
  long long sy, sz, sv;
  double tol, cvd;                     // c_vd = R_d / (gamma - 1)
  double sigma[MAX_TRACERS];           // heat capacities over c_vd
  double mu[MAX_TRACERS];              // chemical potentials (J/kg)
  SatAdjSpec s[MAX_TRACERS / 2];
};

struct SumArgs {
  int nx, ny, nz, gy, nvar;
  long long sy, sz, sv;
  int pert;                       // perturbation storage: add rhobar_k and pbar_k / (gamma - 1)
  double inv_gm1;
  const double* rbar_c;           // nz + 6 (read only with pert)
  const double* pbar_c;
};

// Tile shape of the stage kernels for an element size and variable count.
struct TileShape {
  int tx, ty;
};
TileShape tile_f64(int nv);
TileShape tile_f32(int nv);
int occupancy_f64(int ntracer, bool d3);
int occupancy_f32(int ntracer, bool d3);
int occupancy_mix_f64(int ntracer, bool d3);
int occupancy_mix_f32(int ntracer, bool d3);
int occupancy_hllc_f64(int ntracer, bool d3);
int occupancy_hllc_f32(int ntracer, bool d3);

struct AdjArgs;

// Workspace pointers of one right-hand-side adjoint.
struct AdjWork {
  void* P;   // padded primitive cotangent
};

// Launchers; each returns 0 on success, -1 if the launch failed.
int launch_adj_rhs_f64(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                       void* out, int mode, double alpha, double beta, const void* y, double gam,
                       hipStream_t st);
int launch_adj_rhs_f32(const AdjWork& w, const AdjArgs& a, const void* q, const void* rb,
                       void* out, int mode, double alpha, double beta, const void* y, double gam,
                       hipStream_t st);
int launch_stage_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
// The stage kernels without tracers (LMARS, or HLLC with hllc = true) live in
// translation units of their own, compiled with another instruction scheduling
// strategy than the kernels with tracers (see build.py).
int launch_stage_dry_f64(bool hllc, bool d3, const StageArgs& a, int nblocks, hipStream_t st);
int launch_stage_dry_f32(bool hllc, bool d3, const StageArgs& a, int nblocks, hipStream_t st);
int occupancy_dry_f64(bool hllc, bool d3);
int occupancy_dry_f32(bool hllc, bool d3);
int launch_stage_f32(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
int launch_stage_mix_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
int launch_stage_mix_f32(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
// 3-D mixture kernels with the sedimentation terms (falling condensates).
int launch_stage_sed_f64(int ntracer, const StageArgs& a, int nblocks, hipStream_t st);
int launch_stage_sed_f32(int ntracer, const StageArgs& a, int nblocks, hipStream_t st);
int occupancy_sed_f64(int ntracer);
int occupancy_sed_f32(int ntracer);
int launch_stage_hllc_f64(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
int launch_stage_hllc_f32(int ntracer, bool d3, StageArgs a, int nblocks, hipStream_t st);
int launch_fill_ghosts(int dtype, void* q, const GhostArgs& a, hipStream_t st);
int launch_fill_ghosts_batched(int dtype, const GhostDesc* d, int n, long long max_ghosts,
                               hipStream_t st);

// Batched (ensemble) 2-D stage kernel: tile variant v of the element type.
constexpr int BATCH_VARIANTS = 6;
TileShape batched_tile(int dtype, int ntracer, int variant);   // {0, 0}: unavailable
// form: 0 passive tracers with LMARS, 1 the mixture equation of state, 2 HLLC
int batched_occupancy(int dtype, int ntracer, int variant, int form);
int launch_stage2d_batched(int dtype, int ntracer, int variant, int form, const StageArgs* descs,
                           const int* first, int n, int nblocks, hipStream_t st);
int launch_cfl(int dtype, const void* q, const CflArgs& a, unsigned long long* out,
               hipStream_t st);
int launch_kessler(int dtype, int ntracer, void* q, const KesslerArgs& a, hipStream_t st);
int launch_kessler_adj(int dtype, int ntracer, const void* q, void* qb, const KesslerArgs& a,
                       hipStream_t st);
int launch_satadj(int dtype, int ntracer, void* q, const SatAdjArgs& a, hipStream_t st);
int launch_satadj_adj(int dtype, int ntracer, const void* q, void* qb, const SatAdjArgs& a,
                      hipStream_t st);
int launch_sediment(int dtype, int ntracer, const StageArgs& a, hipStream_t st);
int launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
int launch_flag_speed(const unsigned long long* smax, unsigned long long* flag, hipStream_t st);
int launch_sums(int dtype, const void* q, const SumArgs& a, double* part, double* out,
                hipStream_t st);

}  // namespace snap
