/*
 * libsnap: C-ABI of the SNAP finite-volume hot path on AMD Instinct MI355X (gfx950).
 *
 * The library advances the compressible Euler equations with total energy as
 * the prognostic variable and passive tracer densities (Li & Chen, "Simulating
 * Non-hydrostatic atmospheres on Planets", Sec. 2 and App. B): a conserved state
 * Y = (rho, rho u, rho v, rho w, E, rho_1 .. rho_NT) on a collocated structured
 * grid (Sec. 4, eq. forward), fifth-order WENO reconstruction of primitive
 * variables at cell faces (Sec. 4.2, eq. weno5), the LMARS face flux (Sec. 4.1,
 * eqs. rp and ru), the flux divergence and the gravity body force (Sec. 4, eq.
 * forward), and the three-stage TVD Runge-Kutta step (Sec. 4.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers are DEVICE pointers unless an argument is documented as host memory.
 * The caller owns and allocates every buffer; the library never allocates or
 * frees device memory. Scratch memory comes in through `work`, sized by
 * snap_workspace_bytes() for the matching operation.
 *
 * State layout: q[nvar][nz + 2 ng][ny + 2 gy][nx + 2 ng], x fastest, ng = 3
 * ghost layers (the six-cell face stencil of the fifth-order reconstruction,
 * Sec. 4, stencil equations for Q- and Q+ with m = 3), gy = ng for 3-D and
 * gy = 0 when ny == 1 (2-D x-z problems have no y ghosts and no y sweep).
 * Field order: rho, rho*u, rho*v, rho*w, E, then ntracer tracer densities.
 * Element type: double for SNAP_F64, float for SNAP_F32.
 *
 * Ghost layers of q are library scratch: a call that reads q either fills them
 * from the interior according to `bc` or reads each ghost value at the
 * interior cell it copies (the 3-D time-stepping calls without tracers), and
 * leaves them unspecified. Interior cells of q are read-only except in the
 * time-stepping and microphysics calls.
 *
 * Calls are asynchronous on `stream` (a hipStream_t, NULL = default stream),
 * except snap_cfl_dt, snap_conservation_sums(_noalloc) and
 * snap_rk3_steps_status, which return host values and synchronise that
 * stream. Validation of every argument happens on the host
 * before any HIP call: an invalid call returns SNAP_E_INVALID and touches no
 * device state. A failed HIP call returns SNAP_E_DEVICE. The message of the
 * last error of the calling thread is returned by snap_last_error().
 */
#ifndef SNAP_H
#define SNAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNAP_ABI_VERSION 13

/* return codes */
#define SNAP_OK 0
#define SNAP_E_INVALID (-1)     /* bad argument, detected on the host before any HIP call */
#define SNAP_E_UNSUPPORTED (-2) /* e.g. ntracer > SNAP_MAX_TRACERS */
#define SNAP_E_DEVICE (-3)      /* a HIP launch or runtime call failed */
#define SNAP_E_STATE (-4)       /* non-finite or non-positive density or pressure found */

/* element types */
#define SNAP_F64 0
#define SNAP_F32 1

/* boundary conditions per axis */
#define SNAP_BC_PERIODIC 0 /* ghost cell i takes interior cell i mod n */
#define SNAP_BC_REFLECT 1  /* mirror of the conserved state, normal momentum negated */

#define SNAP_NG 3
#define SNAP_MAX_TRACERS 8

/* Riemann solver at the faces */
#define SNAP_RIEMANN_LMARS 0 /* Sec. 4.1 (what a zero-initialised struct selects) */
#define SNAP_RIEMANN_HLLC 1  /* HLLC with Davis wave speeds (passive tracers only) */

/* equation of state */
#define SNAP_EOS_PASSIVE 0 /* tracers do not enter the pressure */
#define SNAP_EOS_MIXTURE 1 /* ideal-gas mixture with condensates (Sec. 2, App. B) */

/* storage form of the state q */
#define SNAP_STORE_TOTAL 0        /* the conserved state of App. B (what a zero-initialised struct selects) */
#define SNAP_STORE_PERTURBATION 1 /* rho - rhobar_k and E - pbar_k / (gamma - 1) in place of rho and E */

/* tracer kinds under SNAP_EOS_MIXTURE */
#define SNAP_TRACER_VAPOUR 0     /* a gas: partial pressure rho_i R_d T / eps_i */
#define SNAP_TRACER_CONDENSATE 1 /* mass and heat capacity, no partial pressure */

/* operations for snap_workspace_bytes */
#define SNAP_OP_RHS 0
#define SNAP_OP_RK3 1
#define SNAP_OP_CFL 2
#define SNAP_OP_SUMS 3
#define SNAP_OP_RHS_ADJ 4
#define SNAP_OP_RK3_ADJ 5
#define SNAP_OP_RK3_CFL 6

/*
 * Grid, physical constants and hydrostatic reference profiles.
 *
 * nx, ny, nz     interior cells, each >= 1; ny == 1 selects a 2-D x-z problem.
 * ng             must be SNAP_NG.
 * ntracer        tracer densities, 0 .. SNAP_MAX_TRACERS; nvar = 5 + ntracer.
 *                Under SNAP_EOS_PASSIVE they do not enter the equation of state:
 *                with no condensate mass and vapour heat capacities in the ratio
 *                of their gas constants the mixture relation of App. B reduces
 *                to p = (gamma - 1)(E - K).
 * dtype          SNAP_F64 or SNAP_F32 element type of q, rhs and work.
 * bc[3]          boundary condition of the x, y and z axes (bc[1] ignored in 2-D).
 * weno_linear    1 = linear weights (0.1, 0.6, 0.3) of Sec. 4.2 (fifth-order
 *                polynomial reconstruction), 0 = nonlinear Jiang-Shu weights.
 * dx, dy, dz     cell sizes in metres, > 0 (dy ignored in 2-D).
 * gamma          ratio of specific heats, > 1.
 * grav           gravitational acceleration >= 0, acting along -z.
 * weno_eps       regulariser of the nonlinear weights, in [1e-30, 1e30] (1e-6 is
 *                customary).
 * rhobar_cell,   DEVICE, nz + 2 ng doubles each: reference density and pressure
 * pbar_cell      of every level, ghost levels included (the caller mirrors them
 *                for a reflecting z axis and wraps them for a periodic one).
 * rhobar_face,   DEVICE, nz + 1 doubles each: reference density and pressure at
 * pbar_face      the z faces; index k is the face between levels k-1 and k.
 * eos            SNAP_EOS_PASSIVE (0; what a zero-initialised struct selects) or
 *                SNAP_EOS_MIXTURE. With the mixture (App. B, eq. p2 and the
 *                effective adiabatic index; gamma is then gamma_d of the dry gas)
 *                tracer t of kind tracer_kind[t] has:
 *                  a_t = 1/tracer_eps[t] - 1 (vapour) or -1 (condensate),
 *                  b_t = tracer_sigma[t] - 1, chemical potential tracer_mu[t],
 *                and with q_t = rho_t / rho, A = sum mu_t rho_t:
 *                  p = (gamma - 1) (1 + sum a_t q_t) / (1 + sum b_t q_t) (E - K - A);
 *                the same ratio of the face mass fractions gives each side of a
 *                face its effective gamma (sound speed) and internal energy.
 * tracer_eps     molar mass of a vapour over that of the dry gas, finite > 0
 *                (ignored for condensates).
 * tracer_sigma   heat capacity at constant volume of a vapour (of a condensate:
 *                its heat capacity) over c_v of the dry gas, finite > 0.
 * tracer_mu      chemical potential per unit mass, J/kg, finite (0 for gases
 *                whose potentials are set to zero; for a condensate
 *                mu_i - (L^r + (c_ij - c_p,i) T^r), Sec. 2, eq. muij).
 * tracer_wt      sedimentation (Sec. 2, eq. d3, the momentum and total-energy
 *                equations): signed vertical velocity (m/s) of condensate t
 *                relative to the air, negative when it falls; 0 for no fall
 *                (and for every vapour). Through every z face a falling
 *                condensate carries the mass flux m = w_t rho_t (into rho_t and
 *                the total density), the momentum m (u, v, w) and the energy
 *                m (c_t T + |u|^2 / 2 + mu_t), c_t = tracer_sigma[t] rd /
 *                (gamma - 1), T = p / (rd rho (1 + sum a_s q_s)); the face value
 *                is that of the cell the condensate comes from (first-order
 *                upwind; the paper gives no discretisation); a reflecting z
 *                boundary lets no condensate in and lets it out (precipitation
 *                leaves through the ground). Its weight heats the air by
 *                -g rho_t w_t. The CFL step does not include |w_t|.
 * rd             gas constant of the dry gas (J/kg/K), finite > 0 when any
 *                tracer_wt is nonzero; not read otherwise.
 * riemann        SNAP_RIEMANN_LMARS or SNAP_RIEMANN_HLLC, the flux at every face.
 *                HLLC: Davis outer wave speeds, contact speed S*, star states
 *                U*_K = rho_K (S_K - u_K)/(S_K - S*) (1, S* / tangential
 *                velocities, E_K/rho_K + (S* - u_K)(S* + p_K / (rho_K (S_K - u_K))),
 *                q_K), with full face density and pressure; the normal momentum
 *                flux carries the perturbation pressure as under LMARS. HLLC
 *                takes eos = SNAP_EOS_PASSIVE. The adjoint entry points take
 *                either flux.
 *                The tracer fields are read only under SNAP_EOS_MIXTURE with
 *                ntracer > 0 (a nonzero tracer_wt needs the mixture). The
 *                adjoint entry points take the mixture and falling condensates
 *                (the reverse of the sedimentation terms).
 * storage        SNAP_STORE_TOTAL (0): q holds the conserved state.
 *                SNAP_STORE_PERTURBATION: q[0] holds rho - rhobar_k and q[4]
 *                holds E - pbar_k / (gamma - 1) (the state's departure from the
 *                reference level k at rest; ghost levels use the ghost-level
 *                references), the other fields as in SNAP_STORE_TOTAL. Every
 *                entry point takes and returns q in this form; the right-hand
 *                side, cotangents and time steps are those of the full state
 *                (the stage combination of Sec. 4.3 has weights summing to one,
 *                so the references cancel), and the conservation sums are of
 *                the full fields. With single-precision storage this keeps the
 *                digits of the departure that rounding the full E (about
 *                2.5e5 J/m^3 near the ground) to FP32 would lose. Passive
 *                tracers only: with SNAP_EOS_MIXTURE it returns
 *                SNAP_E_UNSUPPORTED.
 *
 * Density and pressure are reconstructed as perturbations rho - rhobar and
 * p - pbar of the level (the vertical perturbation pressure of Sec. 4.1); face
 * values add back the face reference on z faces and the level reference on x
 * and y faces. The gravity source is -g (rho - rhobar_k) on vertical momentum
 * and -g rho w on energy, which equals the full-pressure form when rhobar_k is
 * the discretely hydrostatic (pbar_{k-1/2} - pbar_{k+1/2}) / (g dz).
 */
typedef struct snap_grid {
  int32_t nx, ny, nz;
  int32_t ng;
  int32_t ntracer;
  int32_t dtype;
  int32_t bc[3];
  int32_t weno_linear;
  double dx, dy, dz;
  double gamma, grav;
  double weno_eps;
  const double* rhobar_cell;
  const double* pbar_cell;
  const double* rhobar_face;
  const double* pbar_face;
  int32_t eos;
  int32_t tracer_kind[SNAP_MAX_TRACERS];
  double tracer_eps[SNAP_MAX_TRACERS];
  double tracer_sigma[SNAP_MAX_TRACERS];
  double tracer_mu[SNAP_MAX_TRACERS];
  double tracer_wt[SNAP_MAX_TRACERS];
  double rd;
  int32_t riemann;
  int32_t storage;
} snap_grid;

/* Thread-local message of the last failed call of this thread ("" if none). */
const char* snap_last_error(void);

/* SNAP_ABI_VERSION of the loaded library. */
int snap_abi_version(void);

/*
 * Bytes of device workspace `work` needed by operation `op` (SNAP_OP_*) on grid
 * g; 0 if none is needed. Returns 0 and sets the last error for an invalid grid.
 * SNAP_OP_RK3 needs two padded state arrays, SNAP_OP_RK3_CFL the same plus
 * 256 bytes (two signal-speed slots and the state flag read by
 * snap_rk3_steps_status), SNAP_OP_RHS_ADJ one padded array, SNAP_OP_RK3_ADJ
 * three padded plus two interior arrays, SNAP_OP_CFL and SNAP_OP_SUMS a few
 * hundred kilobytes of reduction partials.
 */
size_t snap_workspace_bytes(const snap_grid* g, int op);

/*
 * Fill the ghost layers of q (padded layout, dtype of g) from its interior
 * according to g->bc: periodic = wrap copy; reflecting = mirror image of the
 * conserved state with the momentum component normal to the wall negated
 * (boundary conditions named in Sec. 5; the ghost-cell form is this library's
 * reading). Corner ghosts take the composition of the per-axis maps.
 */
int snap_fill_ghosts(const snap_grid* g, void* q, void* stream);

/*
 * Right-hand side of the semi-discrete system (Sec. 4, eq. forward with the
 * Riemann flux of Sec. 4.1 and the reconstruction of Sec. 4.2):
 *   rhs = -sum_d (F_{+1/2} - F_{-1/2}) / dx_d + body force
 * for every interior cell.
 * q    padded state (ghosts overwritten, interior read).
 * rhs  interior array rhs[nvar][nz][ny][nx], x fastest, overwritten.
 */
int snap_rhs(const snap_grid* g, void* q, void* rhs, void* stream);

/*
 * One three-stage TVD Runge-Kutta step (Sec. 4.3) of the full multi-direction
 * right-hand side with a fixed time step dt (host value, finite and > 0):
 *   Q1 = Q + dt R(Q); Q2 = 3/4 Q + 1/4 (Q1 + dt R(Q1));
 *   Q <- 1/3 Q + 2/3 (Q2 + dt R(Q2)).
 * q     padded state: interior in = Q^n, interior out = Q^{n+1}; ghost layers on
 *       return are unspecified (snap_fill_ghosts refreshes them).
 * work  device workspace of snap_workspace_bytes(g, SNAP_OP_RK3) bytes; on
 *       return it holds the stage states Q1 and Q2 (interiors; see
 *       snap_rk3_step_adjoint_stages for the layout).
 */
int snap_rk3_step(const snap_grid* g, void* q, double dt, void* work, void* stream);

/*
 * Discrete adjoint of the right-hand side (reverse mode of snap_rhs, i.e. of
 * Sec. 4 eq. forward with the fluxes of Sec. 4.1 and the reconstruction of
 * Sec. 4.2, ghost cells being functions of the interior through `bc`):
 *   q_bar = J(q)^T rhs_bar,  J = d rhs / d (interior of q).
 * q        padded state at which J is taken (ghosts overwritten, interior read).
 * rhs_bar  interior array [nvar][nz][ny][nx], read.
 * q_bar    interior array [nvar][nz][ny][nx], overwritten; must not alias q or
 *          rhs_bar.
 * At an interface velocity u* of exactly zero, where the upwind choice of LMARS
 * switches sides, the derivative of the advective flux with respect to u* uses
 * the mean of both sides' advected vectors (the one-sided derivatives differ
 * there). With HLLC the derivative is that of the branch (side, star region)
 * and of the outer wave speed candidates the forward evaluation selects. With
 * falling condensates the sedimentation terms (upwind fall fluxes through the
 * z faces and the frictional heating) are reversed as well, each face's flux
 * being a function of its source cell. The result is reproducible bit for bit
 * (no atomics).
 * work  device workspace of snap_workspace_bytes(g, SNAP_OP_RHS_ADJ) bytes.
 */
int snap_rhs_adjoint(const snap_grid* g, void* q, const void* rhs_bar, void* q_bar, void* work,
                     void* stream);

/*
 * Adjoint of one snap_rk3_step with the same fixed dt (dt is not a variable of
 * differentiation): given q_bar = dL/dQ^{n+1}, overwrite it with dL/dQ^n.
 * The stage states Q1 and Q2 are recomputed from q_n; then, reversing the
 * three stages of Sec. 4.3,
 *   B2 = 2/3 (q_bar + dt J(Q2)^T q_bar);  B1 = 1/4 (B2 + dt J(Q1)^T B2);
 *   q_bar <- q_bar/3 + 3/4 B2 + B1 + dt J(Q^n)^T B1.
 * q_n    padded state Q^n (ghosts overwritten, interior read).
 * q_bar  interior array [nvar][nz][ny][nx], in: dL/dQ^{n+1}, out: dL/dQ^n.
 * work   device workspace of snap_workspace_bytes(g, SNAP_OP_RK3_ADJ) bytes.
 */
int snap_rk3_step_adjoint(const snap_grid* g, void* q_n, double dt, void* q_bar, void* work,
                          void* stream);

/*
 * snap_rk3_step_adjoint with the stage states kept from the forward step
 * instead of recomputed (Sec. 4.3, the same reverse of the three stages):
 * two stage kernels fewer per step, for callers that can hold the stage states
 * of every step they walk back through (two padded states per step).
 * stages  the workspace (SNAP_OP_RK3) of the snap_rk3_step call that advanced
 *         Q^n with this dt: on return snap_rk3_step leaves Q1 in its first
 *         padded block and Q2 in the block that starts at the first multiple
 *         of 256 bytes past it. Their ghost cells are overwritten here, their
 *         interiors read; the step must not have been followed by another
 *         call that uses the same workspace.
 * q_n, q_bar, work, errors: as for snap_rk3_step_adjoint (work of
 *         snap_workspace_bytes(g, SNAP_OP_RK3_ADJ) bytes, of which the first
 *         two padded blocks go unused); SNAP_E_INVALID if stages is NULL.
 */
int snap_rk3_step_adjoint_stages(const snap_grid* g, void* q_n, void* stages, double dt,
                                 void* q_bar, void* work, void* stream);

/*
 * Largest stable step dt = cfl / max over interior cells of
 *   sum_d (|u_d| + c) / dx_d,  c = sqrt(gamma p / rho)
 * (the time-step rule is this library's reading; the paper gives none).
 * dt_host  HOST pointer receiving dt. The call synchronises `stream`.
 * Returns SNAP_E_STATE (and leaves *dt_host untouched) if any interior cell has
 * a non-finite or non-positive density or pressure.
 * work  device workspace of snap_workspace_bytes(g, SNAP_OP_CFL) bytes.
 */
int snap_cfl_dt(const snap_grid* g, void* q, double cfl, void* work, double* dt_host, void* stream);

/*
 * snap_cfl_dt followed by snap_rk3_step, with dt kept on the device: the
 * maximum signal speed of Q^n is reduced into `work`, and each stage kernel
 * forms dt = cfl / (that maximum) itself, the same double division the host
 * makes in snap_cfl_dt, so the step equals snap_rk3_step with that dt bit for
 * bit. The host neither waits for nor needs dt: steps can be queued back to
 * back (and captured in a graph, no memset being recorded).
 * q       padded state, as in snap_rk3_step.
 * cfl     host value, finite and > 0.
 * work    device workspace of snap_workspace_bytes(g, SNAP_OP_RK3_CFL) bytes.
 * dt_dev  DEVICE pointer receiving the step's dt (one double), or NULL.
 * Argument errors are reported as by snap_rk3_step. A state that snap_cfl_dt
 * would reject (non-finite or non-positive density or pressure) gives a dt and
 * new states that are not finite; the call does not wait to report it, but it
 * leaves a flag in `work` that snap_rk3_steps_status turns into SNAP_E_STATE.
 */
int snap_rk3_step_cfl(const snap_grid* g, void* q, double cfl, void* work, double* dt_dev,
                      void* stream);

/*
 * nsteps calls of snap_rk3_step_cfl in one: the same steps, bit for bit, each
 * taking dt = cfl / (maximum signal speed of its Q^n). For 3-D grids without
 * tracers (or sedimentation) the last stage of each step also
 * reduces the signal speed of the state it writes, so the next step needs no
 * separate reduction pass over Q^n.
 * nsteps  >= 1.
 * work    device workspace of snap_workspace_bytes(g, SNAP_OP_RK3_CFL) bytes.
 * dt_dev  DEVICE pointer receiving the nsteps time steps (doubles), or NULL.
 * Errors as for snap_rk3_step_cfl, and SNAP_E_INVALID for nsteps < 1.
 */
int snap_rk3_steps_cfl(const snap_grid* g, void* q, double cfl, int nsteps, void* work,
                       double* dt_dev, void* stream);

/*
 * State check of the last snap_rk3_step_cfl / snap_rk3_steps_cfl call that
 * used `work` (a SNAP_OP_RK3_CFL workspace of grid g): synchronises `stream`
 * and returns SNAP_E_STATE if the state that any step of that call started
 * from had a non-finite or non-positive density or pressure somewhere (the
 * CFL reduction of that state, Sec. 4.3's time step being this library's
 * reading, is then NaN, and so are its dt and every later state), else
 * SNAP_OK. On 3-D grids without tracers (whose last stage reduces the signal
 * speed of the state it writes) the state the call ends with is checked too;
 * on other grids that state is checked by the next step or by snap_cfl_dt.
 * The flag is cleared by each device-dt call, not by this one; reading it
 * costs one 8-byte copy. The result is undefined for a workspace that no such
 * call has used.
 */
int snap_rk3_steps_status(const snap_grid* g, void* work, void* stream);

/*
 * Sums over interior cells of every conserved field, accumulated in double
 * precision in a fixed order (mass and total energy are conserved by the
 * flux form, Sec. 4, eq. forward).
 * sums_host  HOST array of nvar doubles. The call synchronises `stream`.
 * work  device workspace of snap_workspace_bytes(g, SNAP_OP_SUMS) bytes.
 */
int snap_conservation_sums(const snap_grid* g, void* q, void* work, double* sums_host, void* stream);

/*
 * snap_conservation_sums without a workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The call allocates nothing: the partial
 * sums live in a library-owned device array of SNAP_SUMS_NOALLOC_SCRATCH_BYTES
 * bytes, which every GPU the library runs on holds (its own copy) until the
 * process ends, and whose address is looked up on the first call on each
 * device. It holds the partials of every valid grid (up to 5 +
 * SNAP_MAX_TRACERS variables); a grid needing more returns SNAP_E_INVALID.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (other streams, other threads) race, and the caller must serialise them.
 * Results equal those of snap_conservation_sums bit for bit; q, sums_host,
 * the synchronisation of `stream` and the errors are as there.
 */
#define SNAP_SUMS_NOALLOC_SCRATCH_BYTES 53760
int snap_conservation_sums_noalloc(const snap_grid* g, void* q, double* sums_host, void* stream);

/*
 * Ensemble of independent 2-D (ny == 1) domains advanced by one SSP-RK3 step
 * each (Sec. 4.3), with per-member grids, states and time steps. Every stage
 * is one batched ghost-fill launch and one persistent stage launch for all
 * members: `nblocks` workgroups walk the (member, tile) work items round-robin
 * (0 = as many as fit on the device at once). Members must share dtype,
 * ntracer, equation of state and Riemann solver (the passive gas or the
 * mixture; LMARS or HLLC), else SNAP_E_INVALID; 3-D members, and members
 * whose condensates fall (the sedimentation of Sec. 2), return
 * SNAP_E_UNSUPPORTED; 1 <= n <= 65535.
 * gs       HOST array of n grids (each with its own DEVICE reference profiles).
 * q        HOST array of n DEVICE pointers to padded member states (in Q^n,
 *          out Q^{n+1}; ghost layers unspecified on return).
 * dt_host  HOST array of n time steps, each finite and > 0.
 * variant  tile shape (snap_batched_tile_variant); 0 is the single-domain
 *          default, 1..5 are alternatives (ntracer == 0 only) for autotuning.
 * work     device workspace of snap_batched_workspace_bytes(gs, n) bytes; it
 *          holds the descriptor tables (copied from the host on each call)
 *          and two stage states per member.
 */
size_t snap_batched_workspace_bytes(const snap_grid* gs, int n);
int snap_batched_tile_variant(int dtype, int ntracer, int variant, int* tx, int* tz);
int snap_rk3_step_batched(const snap_grid* gs, int n, void* const* q, const double* dt_host,
                          int variant, int nblocks, void* work, void* stream);

/*
 * Kessler microphysics (Sec. 3), operator-split after a time step.
 *
 * Per condensable species: the mass mixing ratios X = (q_v, q_c, q_p) of its
 * vapour, cloud and precipitation evolve by
 *   dq_v/dt = -k1 (q_v - q*)+ + k4 q_p (q* - q_v)+
 *   dq_c/dt =  k1 (q_v - q*)+ - k3 q_c q_p - k2 q_c
 *   dq_p/dt = -k4 q_p (q* - q_v)+ + k3 q_c q_p + k2 q_c      (x+ = max(x, 0)),
 * integrated over dt by backward Euler, X = X^n + dt Phi(X), with the Newton
 * iteration of Sec. 3 (eq. x_n+1) started at X^n: rates and Jacobian of the
 * regime of X^n (saturated if q_v > q*; backward Euler keeps q_v on that
 * side of q*); the unsaturated Jacobian includes d/dq_p of the evaporation
 * term, which the printed matrix leaves out (the fixed point does not depend
 * on it). The iteration stops when the largest Newton step is at most
 * tol (q_v + q_c + q_p)^n, or after max_iter steps. It can land on the
 * unphysical root of the accretion quadratic when dt k3 (q_c - q_p) > 1.
 * q* = p*(T) eps / (R_d T rho), with eps the vapour's tracer_eps, the
 * saturation vapour pressure over the cloud p* = p_ref exp[beta (1 - 1/t) -
 * delta ln t], t = T / t_ref (App. D, integrated Clausius-Clapeyron), and the
 * temperature of the mixture T = p / (R_d (rho_d + sum_vapours rho_i / eps_i))
 * (Sec. 2, eq. eos), both taken at the start and held through the step.
 * Afterwards rho_t = rho q_t for the three tracers; total density, momentum
 * and total energy are unchanged (the temperature follows from them through
 * the chemical potentials). The arithmetic is double precision whatever the
 * storage type.
 *
 * g      grid with eos = SNAP_EOS_MIXTURE: vapour tracers of kind
 *        SNAP_TRACER_VAPOUR, cloud and precipitation of kind SNAP_TRACER_CONDENSATE.
 * q      padded state, interior updated in place (ghost layers untouched).
 * dt     finite > 0.
 * k      HOST parameters; nspecies in 1 .. SNAP_KESSLER_MAX_SPECIES, tracer
 *        indices in [0, ntracer) and all distinct; k1..k4 finite >= 0; p_ref,
 *        t_ref, rd finite > 0; beta, delta finite; max_iter in 1 .. 100; tol
 *        finite >= 0.
 * Returns SNAP_E_INVALID for any other input; no workspace is needed.
 */
#define SNAP_KESSLER_MAX_SPECIES (SNAP_MAX_TRACERS / 3)

typedef struct snap_kessler_species {
  int32_t vapour, cloud, precip; /* tracer indices */
  double k1, k2, k3, k4;         /* condensation, autoconversion (1/s); accretion, evaporation (1/s per unit q) */
  double p_ref, t_ref;           /* saturation vapour pressure (Pa) at t_ref (K) */
  double beta, delta;            /* (L^r + dc t_ref) / (R_v t_ref) and dc / R_v, dc = c_cloud - c_p,vapour */
} snap_kessler_species;

typedef struct snap_kessler {
  int32_t nspecies;
  snap_kessler_species species[SNAP_KESSLER_MAX_SPECIES];
  double rd;        /* gas constant of the dry gas, J/kg/K */
  int32_t max_iter; /* Newton steps at most */
  double tol;       /* stop at a step of tol x the species' total mixing ratio */
} snap_kessler;

int snap_kessler_step(const snap_grid* g, void* q, double dt, const snap_kessler* k, void* stream);

/*
 * Adjoint of snap_kessler_step (the discrete adjoint of the microphysics step
 * of Sec. 3 as the step above evaluates it): q_bar <- J^T q_bar, J the
 * Jacobian of the state after the step with respect to the state before it,
 * per interior cell. The regime of X^n and the q*, T of the step's start are
 * held, as in the step; the backward-Euler solution X* enters through the
 * implicit-function derivative dX* = M^-1 (dX^n / dt + dPhi/dq* dq*), M = I/dt
 * - dPhi/dX at X* (the step's Newton matrix at its solution), so the result
 * is the transpose of the step's exact derivative once its iteration has
 * converged. Double-precision arithmetic whatever the storage type.
 *
 * g, dt, k  as for snap_kessler_step (the same validation).
 * q      padded state at the START of the step (interior read; ghost layers
 *        not read).
 * q_bar  interior array [nvar][nz][ny][nx] of the storage type: in, the
 *        cotangent of the state after the step; out, that of the state
 *        before it (overwritten in place); must not alias q.
 * Returns SNAP_E_INVALID for any other input; no workspace is needed.
 */
int snap_kessler_step_adjoint(const snap_grid* g, const void* q, double dt, const snap_kessler* k,
                              void* q_bar, void* stream);

/*
 * Saturation adjustment (App. D), the alternative to the Kessler scheme for
 * instantaneous condensation: every vapour is brought to phase equilibrium
 * with its cloud at constant volume and constant total energy.
 *
 * Per cell and vapour / cloud pair the mass x moved from vapour to cloud
 * (negative: cloud evaporated), -rho_c <= x <= rho_v, solves
 *   (rho_v - x) R_v T(x) = p*(T(x)),  R_v = rd / eps_v,
 * with the saturation vapour pressure over the cloud p* = p_ref exp[beta (1 -
 * 1/t) - delta ln t], t = T / t_ref (App. D), and the temperature of the
 * adjusted composition from the conserved energy (Sec. 2, eqs. energy and eos):
 *   T = (E - K - sum_t mu_t rho_t) / (c_vd (rho_d + sum_t sigma_t rho_t)),
 *   c_vd = rd / (gamma - 1);
 * if the vapour stays below saturation with all cloud evaporated, x = -rho_c.
 * The pairs interact through T: each sweep takes, pair by pair, one Newton
 * step on the residual above with the latent heating in its derivative
 * (dT/dx = L_v / (c_vd (rho_d + sum sigma rho)), L_v the latent heat at
 * constant volume), clipped to the limits; the sweeps stop when no step
 * exceeds tol times its pair's total density, or after max_iter sweeps. The
 * paper's own update (eq. dxf with the isochoric alpha) is a Newton-like step
 * on the same condition in molar mixing ratios with an approximate
 * derivative; both have the same fixed point. Total density, momentum and
 * total energy are unchanged; the arithmetic is double precision whatever
 * the storage type.
 *
 * g      grid with eos = SNAP_EOS_MIXTURE: vapours of kind SNAP_TRACER_VAPOUR,
 *        clouds of kind SNAP_TRACER_CONDENSATE.
 * q      padded state, interior updated in place (ghost layers untouched).
 * s      HOST parameters; nspecies in 1 .. SNAP_SATADJ_MAX_SPECIES, tracer
 *        indices in [0, ntracer) and all distinct; p_ref, t_ref, rd finite
 *        > 0; beta, delta finite; max_iter in 1 .. 100; tol finite >= 0.
 * Returns SNAP_E_INVALID for any other input; no workspace is needed.
 */
#define SNAP_SATADJ_MAX_SPECIES (SNAP_MAX_TRACERS / 2)

typedef struct snap_satadj_species {
  int32_t vapour, cloud;  /* tracer indices */
  double p_ref, t_ref;    /* saturation vapour pressure (Pa) at t_ref (K) */
  double beta, delta;     /* (L^r + dc t_ref) / (R_v t_ref) and dc / R_v, dc = c_cloud - c_p,vapour */
} snap_satadj_species;

typedef struct snap_satadj {
  int32_t nspecies;
  snap_satadj_species species[SNAP_SATADJ_MAX_SPECIES];
  double rd;        /* gas constant of the dry gas, J/kg/K */
  int32_t max_iter; /* sweeps over the pairs at most */
  double tol;       /* stop when no step exceeds tol x its pair's total density */
} snap_satadj;

int snap_saturation_adjust(const snap_grid* g, void* q, const snap_satadj* s, void* stream);

/*
 * Adjoint of snap_saturation_adjust (App. D): q_bar <- J^T q_bar, J the
 * derivative of the adjusted state with respect to the state before the
 * adjustment, per interior cell. The adjustment is recomputed; at its
 * equilibrium each pair with cloud left satisfies the condition above, and its
 * transfer x enters through the implicit-function derivative of that
 * condition (the pairs coupled through T: a diagonal plus rank-one system,
 * solved in closed form); a pair whose cloud evaporated entirely follows its
 * bound x = -rho_c. The result is the transpose of the exact derivative of the
 * equilibrium once the sweeps have converged. Double-precision arithmetic
 * whatever the storage type.
 *
 * g, s   as for snap_saturation_adjust (the same validation).
 * q      padded state BEFORE the adjustment (interior read; ghost layers not
 *        read).
 * q_bar  interior array [nvar][nz][ny][nx] of the storage type: in, the
 *        cotangent of the adjusted state; out, that of the state before it
 *        (overwritten in place); must not alias q.
 * Returns SNAP_E_INVALID for any other input; no workspace is needed.
 */
int snap_saturation_adjust_adjoint(const snap_grid* g, const void* q, const snap_satadj* s,
                                   void* q_bar, void* stream);

/*
 * Benchmark instrumentation of the fused stage kernel (the kernel that
 * evaluates the right-hand side and applies one Runge-Kutta stage).
 * snap_stage_timing_enable(1) discards earlier records and brackets every later
 * stage-kernel launch with two hipEvents recorded on the launch stream;
 * snap_stage_timing_enable(0) stops recording. snap_stage_timing_read waits for
 * the recorded events and returns, in HOST memory, the summed duration in
 * milliseconds and the number of timed launches. Process-wide, thread-safe.
 */
int snap_stage_timing_enable(int enable);
int snap_stage_timing_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SNAP_H */
