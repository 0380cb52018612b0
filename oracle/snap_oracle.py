"""Plain FP64 CPU oracle for the SNAP finite-volume right-hand side.

TEST INFRASTRUCTURE ONLY. This module is the correctness reference for the
HIP library: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import it. It shares no code with the GPU path; the two
meet only in the seeded inputs of the ``workloads`` module.

It is written for readability, not speed: whole-array torch CPU operations in
float64 (so that torch autograd yields the discrete adjoint), each step in
the order the paper gives it:

1. ghost cells from the boundary conditions (Sec. 5 names a solid lower
   boundary and doubly periodic domains; the ghost-cell form is the reading
   below);
2. conserved -> primitive variables per cell (App. B, single-gas reduction
   with passive tracers, gamma = gamma_d);
3. per direction, fifth-order WENO reconstruction of the left and right face
   states from primitive variables (Sec. 4.2, eq. weno5 and the stencil
   equations for Q-/Q+ with m = 3), pressure and density reconstructed as
   perturbations from the hydrostatic reference (Sec. 4.1);
4. per face, the LMARS flux (Sec. 4.1, eqs. rp and ru);
5. flux divergence and gravity body force (Sec. 4, eq. forward; Sec. 2,
   momentum and total-energy equations);
6. the three-stage TVD Runge-Kutta step (Sec. 4.3).

Readings of points the paper leaves open (each also listed in the design
notes of the repository):

* WENO nonlinear weights: the classic Jiang-Shu form the paper cites,
  alpha_k = d_k / (eps + beta_k)^2 with the Jiang-Shu smoothness
  indicators; eps is an input (default 1e-6).
* Reconstructed variables in every direction: rho' = rho - rhobar_k, u, v,
  w, p' = p - pbar_k and tracer mass fractions; face values restore
  rho = rhobar_f + rho', p = pbar_f + p' with the face reference for
  z faces and the level reference for x/y faces.
* LMARS averages: rho c -> (rho- + rho+)/2 * (c- + c+)/2, with c = sqrt(gamma p / rho)
  from full face pressure and density.
* LMARS pressure: perturbation pressure in every direction (for x/y faces
  the level reference cancels exactly in the divergence); momentum source
  -g (rho - rhobar_k), equal to -rho g plus the divergence of the
  reference face pressure because rhobar_k is discretely hydrostatic.
* LMARS upwinding: the advected vector (rho, rho u, rho v, rho w, E + p,
  rho q) is taken from the left state when u* > 0, the right state when
  u* < 0, and the mean of both when u* == 0.
* Boundaries: periodic = wrap copy; reflecting = mirror of the conserved
  state with the normal momentum negated.
* Tracers are passive, p = (gamma - 1)(E - K), unless the grid selects the
  mixture equation of state (App. B, eq. p2 and the effective adiabatic
  index): tracer t is a vapour (a_t = 1/eps_t - 1) or a condensate
  (a_t = -1), b_t = sigma_t - 1, A = sum mu_t rho_t, and
  p = (gamma_d - 1) (1 + sum a_t q_t) / (1 + sum b_t q_t) (E - K - A);
  at a face the same ratio with the face's mass fractions gives the
  effective gamma of the sound speed and the internal energy p / (gamma - 1).
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np
import torch

F64 = torch.float64
G = 3
BC_PERIODIC = 0
BC_REFLECT = 1


def _t(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(F64)
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=F64)


def _gy(grid) -> int:
    return 0 if grid.ny == 1 else G


def _axes(grid):
    """Active sweep directions as (array axis, velocity component, spacing, bc, n).

    Array axes of a field are (z, y, x) = (0, 1, 2). The y direction is
    skipped for 2-D x-z problems (ny == 1).
    """
    out = [(2, 0, grid.dx, grid.bc[0], grid.nx)]
    if grid.ny > 1:
        out.append((1, 1, grid.dy, grid.bc[1], grid.ny))
    out.append((0, 2, grid.dz, grid.bc[2], grid.nz))
    return out


# ---------------------------------------------------------------------------
# Boundary conditions
# ---------------------------------------------------------------------------

def fill_ghosts(q: torch.Tensor, grid) -> torch.Tensor:
    """Return a copy of the padded state with all ghost layers filled.

    Periodic: ghost cell i takes the value of interior cell i mod n.
    Reflecting: ghost cell at distance m outside a wall takes the value of
    the interior cell at distance m inside it, with the momentum component
    normal to the wall negated.
    """
    q = _t(q)
    for arr_axis, comp, _, bc, n in _axes(grid):
        ax = arr_axis + 1                       # axis in q (field axis first)
        size = q.shape[ax]
        g = (size - n) // 2
        src = list(range(size))
        sign = torch.ones(size, dtype=F64)
        for m in range(g):
            lo, hi = g - 1 - m, g + n + m
            if bc == BC_PERIODIC:
                src[lo] = g + (n - 1 - m) % n
                src[hi] = g + m % n
            else:
                src[lo] = g + min(m, n - 1)
                src[hi] = g + max(n - 1 - m, 0)
                sign[lo] = -1.0
                sign[hi] = -1.0
        idx = torch.tensor(src, dtype=torch.long)
        q = torch.index_select(q, ax, idx)
        if bc == BC_REFLECT:
            shp = [1] * q.dim()
            shp[ax] = size
            s = sign.reshape(shp)
            normal = q[1 + comp:2 + comp] * s
            q = torch.cat([q[:1 + comp], normal, q[2 + comp:]], dim=0)
    return q


# ---------------------------------------------------------------------------
# Thermodynamics (App. B)
# ---------------------------------------------------------------------------

def mixture_coefficients(grid):
    """(a_t, b_t, mu_t) of every tracer for the mixture equation of state
    (App. B), or None when the tracers are passive.

    a_t: 1/eps_t - 1 for a vapour (molar-mass ratio eps_t), -1 for a
    condensate (it has mass but no partial pressure); b_t = sigma_t - 1 with
    sigma_t the tracer's heat capacity over c_v of the dry gas; mu_t its
    chemical potential per unit mass.
    """
    if getattr(grid, "eos", 0) != 1 or grid.ntracer == 0:
        return None
    coef = []
    for t in range(grid.ntracer):
        a = -1.0 if grid.tracer_kind[t] == 1 else 1.0 / grid.tracer_eps[t] - 1.0
        coef.append((a, grid.tracer_sigma[t] - 1.0, grid.tracer_mu[t]))
    return coef


def mixture_ratio(qs, coef):
    """(1 + sum_t a_t q_t) / (1 + sum_t b_t q_t), summed in tracer order (App. B)."""
    num = 1.0
    den = 1.0
    for qt, (a, b, _) in zip(qs, coef):
        num = num + a * qt
        den = den + b * qt
    return num / den


def cons_to_prim(q: torch.Tensor, grid) -> dict:
    """Primitive variables of every cell of a padded state (App. B).

    The evaluation order is fixed and shared in writing with the GPU path:
    inv = 1/rho; u = (rho u) inv (likewise v, w); K = ((rho u) u + (rho v) v)
    + (rho w) w, times 1/2; p = (gamma - 1)(E - K); p' = p - pbar_k;
    rho' = rho - rhobar_k; q_i = rho_i inv. With the mixture equation of
    state: A = (mu_1 rho_1 + mu_2 rho_2) + ..., num = (1 + a_1 q_1) + ...,
    den likewise, p = ((gamma - 1)(num / den)) ((E - K) - A).
    """
    rho, mx, my, mz, E = q[0], q[1], q[2], q[3], q[4]
    inv = 1.0 / rho
    u = mx * inv
    v = my * inv
    w = mz * inv
    K = 0.5 * ((mx * u + my * v) + mz * w)
    qs = [q[5 + t] * inv for t in range(grid.ntracer)]
    coef = mixture_coefficients(grid)
    if coef is None:
        p = (grid.gamma - 1.0) * (E - K)
    else:
        A = coef[0][2] * q[5]
        for t in range(1, grid.ntracer):
            A = A + coef[t][2] * q[5 + t]
        p = ((grid.gamma - 1.0) * mixture_ratio(qs, coef)) * ((E - K) - A)
    rbar = _t(grid.rhobar_cell).reshape(-1, 1, 1)
    pbar = _t(grid.pbar_cell).reshape(-1, 1, 1)
    prim = {"rho": rho, "u": u, "v": v, "w": w, "p": p,
            "rp": rho - rbar, "pp": p - pbar, "q": qs}
    return prim


def prim_to_cons_energy(rho, u, v, w, p, gamma):
    """Total energy of a single-gas parcel (App. B with A = 0): E = p/(gamma-1) + K."""
    return p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)


# ---------------------------------------------------------------------------
# WENO5 reconstruction (Sec. 4.2)
# ---------------------------------------------------------------------------

LINEAR_WEIGHTS = (0.1, 0.6, 0.3)


def weno5_substencils(a, b, c, d, e):
    """The three third-order candidate values of eq. weno5.

    Arguments are Q_{i-3}, Q_{i-2}, Q_{i-1}, Q_i, Q_{i+1}; the values
    approximate the left state at face i-1/2.
    """
    q0 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c
    q1 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (1.0 / 3.0) * d
    q2 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e
    return q0, q1, q2


def weno5_smoothness(a, b, c, d, e):
    """Jiang-Shu smoothness indicators of the three candidate stencils.

    beta_k is the sum over l = 1, 2 of the integral over the target cell of
    h^(2l-1) (d^l p_k / dx^l)^2 for the quadratic p_k fitted to the cell
    averages of candidate stencil k (the form the paper cites for the
    weights); written out for uniform spacing.
    """
    b0 = (13.0 / 12.0) * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = (13.0 / 12.0) * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = (13.0 / 12.0) * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    return b0, b1, b2


def weno5_weights(a, b, c, d, e, eps: float, linear: bool = False):
    """Normalised convex weights (the paper's alpha_0..alpha_2 of eq. weno5)."""
    if linear:
        one = torch.ones_like(_t(a)) if isinstance(a, torch.Tensor) else 1.0
        return tuple(wk * one for wk in LINEAR_WEIGHTS)
    b0, b1, b2 = weno5_smoothness(a, b, c, d, e)
    a0 = LINEAR_WEIGHTS[0] / (eps + b0) ** 2
    a1 = LINEAR_WEIGHTS[1] / (eps + b1) ** 2
    a2 = LINEAR_WEIGHTS[2] / (eps + b2) ** 2
    s = a0 + a1 + a2
    return a0 / s, a1 / s, a2 / s


def weno5(a, b, c, d, e, eps: float = 1e-6, linear: bool = False):
    """I_weno(Q_{i-3}, Q_{i-2}, Q_{i-1}, Q_i, Q_{i+1}): eq. weno5."""
    q0, q1, q2 = weno5_substencils(a, b, c, d, e)
    w0, w1, w2 = weno5_weights(a, b, c, d, e, eps, linear)
    return w0 * q0 + w1 * q1 + w2 * q2


def reconstruct_faces(v: torch.Tensor, axis: int, n: int, eps: float, linear: bool):
    """Left and right states at the n+1 faces i-1/2 (i = 0..n) along ``axis``.

    ``v`` is padded by G cells on both ends of ``axis``. The left state is
    I(Q_{i-3}, ..., Q_{i+1}) and the right state I(Q_{i+2}, ..., Q_{i-2}),
    the stencil equations of Sec. 4 with m = 3.
    """
    def sl(o):  # Q_{i+o} for i = 0..n, padded index G + i + o
        return v.narrow(axis, G + o, n + 1)
    left = weno5(sl(-3), sl(-2), sl(-1), sl(0), sl(1), eps, linear)
    right = weno5(sl(2), sl(1), sl(0), sl(-1), sl(-2), eps, linear)
    return left, right


# ---------------------------------------------------------------------------
# LMARS (Sec. 4.1)
# ---------------------------------------------------------------------------

def lmars_flux(L: dict, R: dict, normal: int, gamma: float, ntracer: int, thermo=None):
    """LMARS numerical flux at a face from left/right primitive face states.

    Each state holds full density ``rho``, velocity ``u``/``v``/``w``, full
    pressure ``p``, perturbation pressure ``pp`` and tracer mass fractions
    ``q``. Returns the flux of (rho, rho u, rho v, rho w, E, rho q_i).
    ``thermo``: the mixture coefficients of ``mixture_coefficients`` (the
    side's own effective gamma and chemical energy), or None (passive).
    """
    vel = ("u", "v", "w")
    unL, unR = L[vel[normal]], R[vel[normal]]

    def gm1_of(S):   # effective gamma - 1 of a side
        if thermo is None:
            return gamma - 1.0
        return (gamma - 1.0) * mixture_ratio(S["q"], thermo)

    gL, gR = gm1_of(L), gm1_of(R)
    cL = torch.sqrt((1.0 + gL) * L["p"] / L["rho"])
    cR = torch.sqrt((1.0 + gR) * R["p"] / R["rho"])
    rho_avg = 0.5 * (L["rho"] + R["rho"])
    c_avg = 0.5 * (cL + cR)
    rc = rho_avg * c_avg
    pstar = 0.5 * (L["pp"] + R["pp"]) - 0.5 * rc * (unR - unL)      # eq. rp
    ustar = 0.5 * (unL + unR) - (R["pp"] - L["pp"]) / (2.0 * rc)    # eq. ru

    def advected(S, gm1):
        if thermo is None:
            E = prim_to_cons_energy(S["rho"], S["u"], S["v"], S["w"], S["p"], gamma)
        else:   # E = p / (gamma_eff - 1) + K + rho sum mu_t q_t
            E = (S["p"] / gm1 + 0.5 * S["rho"] * (S["u"] ** 2 + S["v"] ** 2 + S["w"] ** 2)
                 + S["rho"] * sum(mu * qt for qt, (_, _, mu) in zip(S["q"], thermo)))
        return ([S["rho"], S["rho"] * S["u"], S["rho"] * S["v"], S["rho"] * S["w"], E + S["p"]]
                + [S["rho"] * qt for qt in S["q"]])

    phiL, phiR = advected(L, gL), advected(R, gR)
    flux = []
    for m, (fl, fr) in enumerate(zip(phiL, phiR)):
        up = torch.where(ustar > 0, fl, torch.where(ustar < 0, fr, 0.5 * (fl + fr)))
        f = ustar * up
        if m == 1 + normal:
            f = f + pstar
        flux.append(f)
    return flux, pstar, ustar


def _conserved_and_flux(S, normal, gamma):
    """Conserved vector U and Euler flux F along ``normal`` of a face state, the
    normal momentum flux with the perturbation pressure (as in LMARS)."""
    vel = [S["u"], S["v"], S["w"]]
    un = vel[normal]
    E = prim_to_cons_energy(S["rho"], S["u"], S["v"], S["w"], S["p"], gamma)
    U = [S["rho"]] + [S["rho"] * vm for vm in vel] + [E] + [S["rho"] * qt for qt in S["q"]]
    F = [S["rho"] * un] + [S["rho"] * vel[m] * un + (S["pp"] if m == normal else 0.0)
                            for m in range(3)]
    F += [(E + S["p"]) * un] + [S["rho"] * qt * un for qt in S["q"]]
    return U, F


def hllc_star(S, Sk, Ss, normal, gamma):
    """Star-region conserved state next to side S (HLLC: the HLL average with the
    contact restored; Toro, Riemann Solvers and Numerical Methods for Fluid
    Dynamics, ch. 10): with un the side's normal velocity and Sk its outer wave
    speed, U* = rho (Sk - un)/(Sk - S*) (1, S* on the normal and the side's
    tangential velocities, E/rho + (S* - un)(S* + p / (rho (Sk - un))), q)."""
    vel = [S["u"], S["v"], S["w"]]
    un = vel[normal]
    E = prim_to_cons_energy(S["rho"], S["u"], S["v"], S["w"], S["p"], gamma)
    fac = S["rho"] * (Sk - un) / (Sk - Ss)
    mom = [fac * (Ss if m == normal else vel[m]) for m in range(3)]
    e = fac * (E / S["rho"] + (Ss - un) * (Ss + S["p"] / (S["rho"] * (Sk - un))))
    return [fac] + mom + [e] + [fac * qt for qt in S["q"]]


def hllc_wave_speeds(L, R, normal, gamma):
    """Outer wave speeds (Davis): S_L = min(u_L - c_L, u_R - c_R),
    S_R = max(u_L + c_L, u_R + c_R); contact speed
    S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R))
         / (rho_L (S_L - u_L) - rho_R (S_R - u_R))."""
    vel = ("u", "v", "w")
    uL, uR = L[vel[normal]], R[vel[normal]]
    cL = torch.sqrt(gamma * L["p"] / L["rho"])
    cR = torch.sqrt(gamma * R["p"] / R["rho"])
    SL = torch.minimum(uL - cL, uR - cR)
    SR = torch.maximum(uL + cL, uR + cR)
    num = R["p"] - L["p"] + L["rho"] * uL * (SL - uL) - R["rho"] * uR * (SR - uR)
    den = L["rho"] * (SL - uL) - R["rho"] * (SR - uR)
    return SL, SR, num / den


def hllc_flux(L: dict, R: dict, normal: int, gamma: float, ntracer: int):
    """HLLC numerical flux at a face (the alternative Riemann solver the paper
    compares LMARS with, Sec. 5): F_L if 0 <= S_L; F_L + S_L (U*_L - U_L) if
    S_L < 0 <= S*; F_R + S_R (U*_R - U_R) if S* < 0 < S_R; F_R if S_R <= 0.
    Face states as for ``lmars_flux``; full pressure and density set the wave
    speeds and star states, and the normal momentum flux carries the
    perturbation pressure (the full flux minus the face reference pressure,
    exact in every branch since the star terms carry no pressure offset).
    Returns (flux, perturbation pressure of the star region, S*)."""
    SL, SR, Ss = hllc_wave_speeds(L, R, normal, gamma)
    UL, FL = _conserved_and_flux(L, normal, gamma)
    UR, FR = _conserved_and_flux(R, normal, gamma)
    sL = hllc_star(L, SL, Ss, normal, gamma)
    sR = hllc_star(R, SR, Ss, normal, gamma)
    flux = []
    for m in range(len(UL)):
        fl_star = FL[m] + SL * (sL[m] - UL[m])
        fr_star = FR[m] + SR * (sR[m] - UR[m])
        flux.append(torch.where(SL >= 0, FL[m], torch.where(Ss >= 0, fl_star,
                                                            torch.where(SR > 0, fr_star, FR[m]))))
    vel = ("u", "v", "w")
    pstar = L["pp"] + L["rho"] * (SL - L[vel[normal]]) * (Ss - L[vel[normal]])
    return flux, pstar, Ss


# ---------------------------------------------------------------------------
# Right-hand side (Sec. 4, eq. forward)
# ---------------------------------------------------------------------------

def _interior_slices(grid, keep_axis: int):
    """Slices selecting interior cells on every array axis except ``keep_axis``."""
    gy = _gy(grid)
    sl = [slice(G, G + grid.nz), slice(gy, gy + grid.ny), slice(G, G + grid.nx)]
    sl[keep_axis] = slice(None)
    return tuple(sl)


def rhs_filled(qf: torch.Tensor, grid) -> torch.Tensor:
    """Right-hand side of the interior cells from a state whose ghosts are filled.

    Returns a tensor of shape (nvar, nz, ny, nx):
    R = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d + body force.
    """
    qf = _t(qf)
    prim = cons_to_prim(qf, grid)
    names = ["rp", "u", "v", "w", "pp"]
    nvar = grid.nvar
    R = [torch.zeros((grid.nz, grid.ny, grid.nx), dtype=F64) for _ in range(nvar)]
    eps, lin = grid.weno_eps, bool(grid.weno_linear)
    for arr_axis, comp, h, _, n in _axes(grid):
        sl = _interior_slices(grid, arr_axis)
        fields = [prim[k][sl] for k in names] + [qt[sl] for qt in prim["q"]]
        rec = [reconstruct_faces(f, arr_axis, n, eps, lin) for f in fields]
        # reference values at the faces of this direction
        if arr_axis == 0:
            rref = _t(grid.rhobar_face).reshape(-1, 1, 1)
            pref = _t(grid.pbar_face).reshape(-1, 1, 1)
        else:
            rref = _t(grid.rhobar_cell)[G:G + grid.nz].reshape(-1, 1, 1)
            pref = _t(grid.pbar_cell)[G:G + grid.nz].reshape(-1, 1, 1)
        states = []
        for side in (0, 1):
            S = {"rho": rref + rec[0][side], "u": rec[1][side], "v": rec[2][side],
                 "w": rec[3][side], "pp": rec[4][side], "p": pref + rec[4][side],
                 "q": [r[side] for r in rec[5:]]}
            states.append(S)
        if getattr(grid, "riemann", 0) == 1:
            flux, _, _ = hllc_flux(states[0], states[1], comp, grid.gamma, grid.ntracer)
        else:
            flux, _, _ = lmars_flux(states[0], states[1], comp, grid.gamma, grid.ntracer,
                                    mixture_coefficients(grid))
        for m in range(nvar):
            F = flux[m]
            dF = F.narrow(arr_axis, 1, n) - F.narrow(arr_axis, 0, n)
            R[m] = R[m] - dF / h
    # gravity along -z: momentum -g (rho - rhobar_k), energy -g (rho w)
    isl = (slice(G, G + grid.nz), slice(_gy(grid), _gy(grid) + grid.ny), slice(G, G + grid.nx))
    R[3] = R[3] - grid.grav * prim["rp"][isl]
    R[4] = R[4] - grid.grav * qf[3][isl]
    if any(getattr(grid, "tracer_wt", ()) or ()):
        _add_sedimentation(qf, grid, prim, R, isl)
    return torch.stack(R)


def _add_sedimentation(qf, grid, prim, R, isl):
    """Sedimentation of condensates (Sec. 2, eqs. d3, the momentum equations
    and the total-energy equation): condensate t with signed vertical velocity
    w_t relative to the air carries, through every z face, the mass flux
    m = w_t rho_t (into rho_t and the total density), the momentum m (u, v, w)
    and the energy m e_t with e_t = c_t T + |u|^2 / 2 + mu_t; its weight does
    the work -g rho_t w_t on the air (energy source).

    Readings: the face value is that of the cell the condensate comes from
    (first-order upwind in the direction of w_t); a reflecting z boundary lets
    no condensate in and lets it out (precipitation leaves through the ground).
    """
    gy = _gy(grid)
    cols = (slice(None), slice(gy, gy + grid.ny), slice(G, G + grid.nx))
    T = temperature(qf, grid, grid.rd)[cols]
    rho = qf[0][cols]
    u, v, w = prim["u"][cols], prim["v"][cols], prim["w"][cols]
    kin = 0.5 * (u * u + v * v + w * w)
    cvd = grid.rd / (grid.gamma - 1.0)
    nz = grid.nz
    closed = grid.bc[2] == BC_REFLECT
    for t, wt in enumerate(grid.tracer_wt):
        if wt == 0.0:
            continue
        rt = qf[5 + t][cols]
        e_t = grid.tracer_sigma[t] * cvd * T + kin + grid.tracer_mu[t]
        # face f (0 .. nz) lies between padded levels G + f - 1 and G + f
        src = slice(G, G + nz + 1) if wt < 0 else slice(G - 1, G + nz)
        m = wt * rt[src]
        per_var = {0: m, 1: m * u[src], 2: m * v[src], 3: m * w[src], 4: m * e_t[src], 5 + t: m}
        for var, F in per_var.items():
            F = F.clone()
            if closed:          # no inflow through a wall
                if wt < 0:
                    F[nz] = 0.0
                else:
                    F[0] = 0.0
            R[var] = R[var] - (F[1:] - F[:-1]) / grid.dz
        R[4] = R[4] - grid.grav * wt * qf[5 + t][isl]


def rhs(q, grid) -> torch.Tensor:
    """Right-hand side (nvar, nz, ny, nx) of a padded state; ghosts filled first."""
    return rhs_filled(fill_ghosts(_t(q), grid), grid)


# ---------------------------------------------------------------------------
# Time stepping (Sec. 4.3)
# ---------------------------------------------------------------------------

def _interior(q, grid):
    gy = _gy(grid)
    return q[:, G:G + grid.nz, gy:gy + grid.ny, G:G + grid.nx]


def _with_interior(q, grid, new_interior):
    gy = _gy(grid)
    out = q.clone()
    out[:, G:G + grid.nz, gy:gy + grid.ny, G:G + grid.nx] = new_interior
    return out


def rk3(rhs_fn: Callable[[torch.Tensor], torch.Tensor], y0: torch.Tensor, dt: float) -> torch.Tensor:
    """Three-stage TVD Runge-Kutta step of Sec. 4.3 for a generic ODE y' = f(y)."""
    y1 = y0 + dt * rhs_fn(y0)
    y2 = 0.75 * y0 + 0.25 * (y1 + dt * rhs_fn(y1))
    return (1.0 / 3.0) * y0 + (2.0 / 3.0) * (y2 + dt * rhs_fn(y2))


def rk3_step(q, grid, dt: float) -> torch.Tensor:
    """One SSP-RK3 step of the padded state; returns the new padded state.

    The ghost layers of the result are filled from its interior.
    """
    q = _t(q)
    qn = _interior(q, grid)

    def f(y_int):
        return rhs(_with_interior(q, grid, y_int), grid)

    new = rk3(f, qn, dt)
    return fill_ghosts(_with_interior(q, grid, new), grid)


def run(q, grid, dt: float, nsteps: int) -> torch.Tensor:
    for _ in range(nsteps):
        q = rk3_step(q, grid, dt)
    return q


# ---------------------------------------------------------------------------
# Time step and diagnostics
# ---------------------------------------------------------------------------

def cfl_dt(q, grid, cfl: float) -> float:
    """dt = cfl / max over interior cells of sum_d (|u_d| + c) / dx_d."""
    q = _interior(_t(q), grid)
    rho = q[0]
    prim = cons_to_prim(q, grid.copy(rhobar_cell=np.zeros(1), pbar_cell=np.zeros(1)))
    u, v, w, p = prim["u"], prim["v"], prim["w"], prim["p"]
    coef = mixture_coefficients(grid)
    gam = grid.gamma if coef is None else 1.0 + (grid.gamma - 1.0) * mixture_ratio(prim["q"], coef)
    c = torch.sqrt(gam * p / rho)
    s = (torch.abs(u) + c) / grid.dx
    if grid.ny > 1:
        s = s + (torch.abs(v) + c) / grid.dy
    s = s + (torch.abs(w) + c) / grid.dz
    bad = ~(rho > 0) | ~(p > 0) | ~torch.isfinite(s)
    if bool(bad.any()):
        raise FloatingPointError("non-positive or non-finite density or pressure")
    return float(cfl / s.max())


def conservation_sums(q, grid) -> np.ndarray:
    """Plain sums over interior cells of every conserved field (float64)."""
    qi = _interior(_t(q), grid)
    return qi.reshape(grid.nvar, -1).sum(dim=1).numpy()


# ---------------------------------------------------------------------------
# Microphysics: Kessler scheme integrated by backward Euler (Sec. 3, App. D)
# ---------------------------------------------------------------------------

def temperature(q, grid, rd: float) -> torch.Tensor:
    """Temperature of every cell of a padded state under the mixture equation
    of state: p = R_d T (rho_d + sum over vapours rho_i / eps_i) (Sec. 2, eq. eos)."""
    q = _t(q)
    p = cons_to_prim(q, grid.copy(rhobar_cell=np.zeros(1), pbar_cell=np.zeros(1)))["p"]
    rho_d = q[0] - sum(q[5 + t] for t in range(grid.ntracer))
    gas = rho_d
    for t in range(grid.ntracer):
        if grid.tracer_kind[t] == 0:
            gas = gas + q[5 + t] / grid.tracer_eps[t]
    return p / (rd * gas)


def saturation_vapour_pressure(T, sp) -> torch.Tensor:
    """p* = p_ref exp[beta (1 - 1/t) - delta ln t], t = T / t_ref (App. D)."""
    t = T / sp.t_ref
    return sp.p_ref * torch.exp(sp.beta * (1.0 - 1.0 / t) - sp.delta * torch.log(t))


def kessler_rates(qv, qc, qp, qs, sp, saturated):
    """Reaction rates of vapour, cloud and precipitation (Sec. 3, eqs. qi .. qi2)
    in the regime ``saturated`` (q_v > q*) or not:
      saturated:   condensation k1 (q_v - q*);
      unsaturated: evaporation k4 q_p (q* - q_v);
      always:      autoconversion k2 q_c and accretion k3 q_c q_p.
    """
    cond = torch.where(saturated, sp.k1 * (qv - qs), torch.zeros_like(qv))
    evap = torch.where(saturated, torch.zeros_like(qv), sp.k4 * qp * (qs - qv))
    conv = sp.k2 * qc + sp.k3 * qc * qp
    return torch.stack([-cond + evap, cond - conv, -evap + conv], dim=-1)


def kessler_jacobian(qv, qc, qp, qs, sp, saturated):
    """d(rates) / d(q_v, q_c, q_p) in the regime ``saturated`` (Sec. 3). The
    unsaturated matrix includes the derivative of evaporation with respect to
    q_p, k4 (q* - q_v), which the printed matrix leaves out; the fixed point of
    the iteration, the backward-Euler solution, does not depend on it."""
    z = torch.zeros_like(qv)
    a = sp.k2 + sp.k3 * qp          # d(conversion)/d q_c
    b = sp.k3 * qc                  # d(conversion)/d q_p
    ev = sp.k4 * (qs - qv)
    rows = [
        [torch.where(saturated, z - sp.k1, -sp.k4 * qp), z, torch.where(saturated, z, ev)],
        [torch.where(saturated, z + sp.k1, z), -a, -b],
        [torch.where(saturated, z, sp.k4 * qp), a, torch.where(saturated, b, b - ev)],
    ]
    return torch.stack([torch.stack(r, dim=-1) for r in rows], dim=-2)


def kessler_solve(qv0, qc0, qp0, qs, sp, dt: float, iters: int = 60):
    """Backward-Euler step X = X^n + dt Phi(X) for X = (q_v, q_c, q_p), by the
    iteration of Sec. 3 (eq. x_n+1): X^{m} = X^{m-1} + (I/dt - J)^{-1}
    [Phi(X^{m-1}) - (X^{m-1} - X^n)/dt], started at X^n. The regime is that
    of X^n: backward Euler keeps q_v on the side of q* it starts on."""
    sat = qv0 > qs
    X0 = torch.stack([qv0, qc0, qp0], dim=-1)
    X = X0.clone()
    eye = torch.eye(3, dtype=F64)
    for _ in range(iters):
        r = kessler_rates(X[..., 0], X[..., 1], X[..., 2], qs, sp, sat) - (X - X0) / dt
        J = kessler_jacobian(X[..., 0], X[..., 1], X[..., 2], qs, sp, sat)
        X = X + torch.linalg.solve(eye / dt - J, r.unsqueeze(-1)).squeeze(-1)
    return X[..., 0], X[..., 1], X[..., 2]


def kessler_step(q, grid, dt: float, kessler) -> torch.Tensor:
    """Padded state after one Kessler microphysics step of length dt.

    Per cell: T from the mixture state, the saturation mixing ratio
    q* = p*(T) eps / (R_d T rho) of each condensable, the backward-Euler
    step of its (vapour, cloud, precipitation) mixing ratios with q* held at
    its value of the step's start, and the new tracer densities rho q. Total
    density, momentum and total energy are unchanged (Sec. 3: rho_d and rho e
    are conserved by phase changes; the temperature follows from them).
    """
    q = _t(q)
    out = q.clone()                 # written; q itself is only read (autograd-safe)
    qi, oi = _interior(q, grid), _interior(out, grid)
    T = _interior(temperature(q, grid, kessler.rd).unsqueeze(0), grid)[0]
    rho = qi[0]
    for sp in kessler.species:
        v, c, pr = 5 + sp.vapour, 5 + sp.cloud, 5 + sp.precip
        qs = saturation_vapour_pressure(T, sp) * sp.eps / (kessler.rd * T) / rho
        qv, qc, qp = kessler_solve(qi[v] / rho, qi[c] / rho, qi[pr] / rho, qs, sp, dt)
        oi[v], oi[c], oi[pr] = rho * qv, rho * qc, rho * qp
    return out


# ---------------------------------------------------------------------------
# Saturation adjustment (App. D): phase equilibrium at constant volume
# ---------------------------------------------------------------------------

def vapour_gas_constant(grid, sp, rd: float) -> float:
    """R_v = R_d / eps_v (eps_v: the vapour's molar mass over the dry gas's)."""
    return rd / grid.tracer_eps[sp.vapour]


def temperature_from_energy(qi, grid, rd: float, ek) -> torch.Tensor:
    """T = (E - K - sum_t mu_t rho_t) / (c_vd (rho_d + sum_t sigma_t rho_t))
    of interior fields qi, given ek = E - K (Sec. 2, eqs. energy and eos)."""
    nt = grid.ntracer
    cvd = rd / (grid.gamma - 1.0)
    a = sum(grid.tracer_mu[t] * qi[5 + t] for t in range(nt))
    c = qi[0] - sum(qi[5 + t] for t in range(nt)) + sum(grid.tracer_sigma[t] * qi[5 + t]
                                                        for t in range(nt))
    return (ek - a) / (cvd * c)


def transfer_bounds(rho_v, rho_c):
    """Limits of the mass moved from vapour to cloud: all cloud evaporated
    (-rho_c) to all vapour condensed (rho_v)."""
    return -rho_c, rho_v.clone()


def saturation_adjust(q, grid, adjust, sweeps: int = 40, bisections: int = 90) -> torch.Tensor:
    """Padded state after saturation adjustment: every vapour brought to phase
    equilibrium with its cloud at constant volume and constant total energy
    (App. D; Sec. 2, eqs. energy and eos for the temperature).

    Plain definition, per cell and vapour / cloud pair: the mass x moved from
    vapour to cloud (negative: cloud evaporated), -rho_c <= x <= rho_v, such
    that the vapour's partial pressure equals the saturation vapour pressure
    at the resulting temperature,
        (rho_v - x) (R_d / eps_v) T(x) = p*(T(x)),
    where T follows from the conserved energy and the new composition,
        T = (E - K - sum_t mu_t rho_t) / (c_vd (rho_d + sum_t sigma_t rho_t));
    if the vapour stays below saturation even with all cloud evaporated,
    x = -rho_c. The residual decreases with x (the vapour pressure falls and
    the latent heat raises p*), so each pair's equation is solved by
    bisection; the pairs interact through the temperature and are swept in
    turn until no transfer changes. Density, momentum and total energy are
    unchanged.
    """
    q = _t(q).clone()
    qi = _interior(q, grid)
    ek = qi[4] - 0.5 * (qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]) / qi[0]
    for _ in range(sweeps):
        moved = 0.0
        for sp in adjust.species:
            v, c = 5 + sp.vapour, 5 + sp.cloud
            rv0, rc0 = qi[v].clone(), qi[c].clone()
            r_vap = vapour_gas_constant(grid, sp, adjust.rd)

            def resid(x):
                qi[v] = rv0 - x
                qi[c] = rc0 + x
                T = temperature_from_energy(qi, grid, adjust.rd, ek)
                return (rv0 - x) * r_vap * T - saturation_vapour_pressure(T, sp)

            lo, hi = transfer_bounds(rv0, rc0)
            f_lo = resid(lo)
            a, b = lo.clone(), hi.clone()
            for _ in range(bisections):
                mid = 0.5 * (a + b)
                above = resid(mid) > 0.0
                a = torch.where(above, mid, a)
                b = torch.where(above, b, mid)
            x = torch.where(f_lo <= 0.0, lo, 0.5 * (a + b))
            qi[v] = rv0 - x
            qi[c] = rc0 + x
            tot = rv0 + rc0
            rel = torch.where(tot > 0, x.abs() / torch.where(tot > 0, tot, torch.ones_like(tot)),
                              torch.zeros_like(tot))
            moved = max(moved, float(rel.max()))
        if moved <= 1e-15:
            break
    return q


def saturation_adjust_diff(q, grid, adjust) -> torch.Tensor:
    """The saturation adjustment (App. D) in a form whose autograd derivative is
    that of the adjusted state with respect to q.

    The bisection of saturation_adjust fixes the transfers X*_s (mass moved
    from vapour s to cloud s) but carries no derivative. At the equilibrium
    every pair with cloud left satisfies G_s(X, q) = 0, with
        G_s = (rho_v,s - X_s) R_v,s T(X, q) - p*_s(T(X, q)),
    T the temperature of the state after the transfers; a pair whose cloud
    evaporated entirely sits on its bound X_s = -rho_c,s. By the implicit
    function theorem dX/dq = -J^{-1} dG/dq over the pairs with cloud left
    (J = dG/dX over those pairs), the bound pairs entering G through T with
    their own derivative. The function returns the state after the transfers
        X = X* - J*^{-1} G(X*, q)   (pairs with cloud left, J* = J at X*, fixed)
        X = -rho_c                 (pairs on the bound),
    whose value is the adjusted state (G(X*) vanishes at convergence) and whose
    derivative is the implicit-function one. Padded layout like q; only the
    species' tracers differ from q.
    """
    q = _t(q)
    with torch.no_grad():
        qa = saturation_adjust(q.detach(), grid, adjust)
    qi = _interior(q, grid)
    qai = _interior(qa, grid)
    ns = len(adjust.species)
    vi = [5 + sp.vapour for sp in adjust.species]
    ci = [5 + sp.cloud for sp in adjust.species]
    rvap = [vapour_gas_constant(grid, sp, adjust.rd) for sp in adjust.species]
    xstar = [(qai[c] - qi[c]).detach() for c in ci]
    bound = [qai[c] <= 0.0 for c in ci]          # cloud evaporated entirely
    ek = qi[4] - 0.5 * (qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]) / qi[0]

    def resid(state, e_k, X):
        new = [state[m] for m in range(state.shape[0])]
        for s in range(ns):
            new[vi[s]] = state[vi[s]] - X[s]
            new[ci[s]] = state[ci[s]] + X[s]
        T = temperature_from_energy(torch.stack(new), grid, adjust.rd, e_k)
        return [(state[vi[s]] - X[s]) * rvap[s] * T
                - saturation_vapour_pressure(T, adjust.species[s]) for s in range(ns)]

    # J* = dG/dX at X*, per cell, by autograd with the state held fixed
    xr = [x.clone().requires_grad_(True) for x in xstar]
    g0 = resid(qi.detach(), ek.detach(), xr)
    rows = []
    for s in range(ns):
        grads = torch.autograd.grad(g0[s].sum(), xr, retain_graph=s + 1 < ns)
        rows.append(torch.stack(grads, dim=-1))
    J = torch.stack(rows, dim=-2)                # (..., s, j)
    act = torch.stack([~b for b in bound], dim=-1)
    both = act.unsqueeze(-1) & act.unsqueeze(-2)
    eye = torch.eye(ns, dtype=F64).expand_as(J)
    Jm = torch.where(both, J, torch.where(act.unsqueeze(-1), torch.zeros_like(J), eye))
    # G at X* (pairs with cloud left) and at the bound (the others), with q live
    xe = [torch.where(bound[s], -qi[ci[s]], xstar[s]) for s in range(ns)]
    g = resid(qi, ek, xe)
    gv = torch.stack([torch.where(bound[s], torch.zeros_like(g[s]), g[s]) for s in range(ns)],
                     dim=-1)
    corr = torch.linalg.solve(Jm.detach(), gv.unsqueeze(-1)).squeeze(-1)
    out = q.clone()
    oi = _interior(out, grid)
    for s in range(ns):
        X = torch.where(bound[s], -qi[ci[s]], xstar[s] - corr[..., s])
        oi[vi[s]] = qi[vi[s]] - X
        oi[ci[s]] = qi[ci[s]] + X
    return out


def saturation_adjust_adjoint(q, grid, adjust, q_bar) -> torch.Tensor:
    """q_bar_in = (d adjusted state / d q)^T q_bar for the interior cells (both
    in the interior layout (nvar, nz, ny, nx)); see saturation_adjust_diff."""
    q = _t(q)
    qi = _interior(q, grid).clone().requires_grad_(True)
    out = saturation_adjust_diff(_with_interior(q.detach(), grid, qi), grid, adjust)
    (g,) = torch.autograd.grad(_interior(out, grid), qi, _t(q_bar))
    return g


# ---------------------------------------------------------------------------
# Discrete adjoint (torch autograd through the oracle)
# ---------------------------------------------------------------------------

def rhs_adjoint(q, grid, rhs_bar) -> torch.Tensor:
    """q_bar = J(q)^T rhs_bar for the interior cells (ghosts folded back).

    Returns a tensor of shape (nvar, nz, ny, nx).
    """
    q = _t(q)
    qi = _interior(q, grid).clone().requires_grad_(True)
    r = rhs(_with_interior(q.detach(), grid, qi), grid)
    (g,) = torch.autograd.grad(r, qi, _t(rhs_bar))
    return g


def rk3_step_adjoint(q, grid, dt: float, q_bar) -> torch.Tensor:
    """dL/dQ^n from dL/dQ^{n+1} (interior arrays) through one RK3 step."""
    q = _t(q)
    qi = _interior(q, grid).clone().requires_grad_(True)
    out = rk3_step(_with_interior(q.detach(), grid, qi), grid, dt)
    (g,) = torch.autograd.grad(_interior(out, grid), qi, _t(q_bar))
    return g
