"""Seeded synthetic workloads for the SNAP finite-volume hot path.

This module is shared by the CPU oracle and by the HIP path (tests and the
benchmark). It holds the grid description, the hydrostatic base states and
the seeded initial conditions, and nothing of the right-hand side itself:
no reconstruction, no Riemann solver, no flux divergence, no time stepping.

State layout (both sides): a float array ``q[nvar][nz+2G][ny+2Gy][nx+2G]``
with x fastest, ``G = 3`` ghost layers (the 6-cell face stencil of the
fifth-order reconstruction, Sec. 4, eqs. for Q-/Q+ with m = 3) and
``Gy = 0`` when ``ny == 1`` (2-D x-z problems carry no y ghosts).
Field order: (rho, rho*u, rho*v, rho*w, E, rho_tracer_1 .. rho_tracer_NT),
the conserved vector of App. B with total density and total energy.

Initial conditions are built from primitive fields with the single-gas
energy relation E = p/(gamma-1) + rho*|u|^2/2 (App. B, passive-tracer
reduction), or, for a grid with the mixture equation of state, from the
species' partial pressures and heat capacities; gravity acts along -z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

G = 3                      # ghost layers
BC_PERIODIC = 0
BC_REFLECT = 1
MAX_TRACERS = 8
RGAS = 8.314462618         # J / (mol K)
RIEMANN_LMARS = 0
RIEMANN_HLLC = 1
EOS_PASSIVE = 0            # tracers do not enter the equation of state
EOS_MIXTURE = 1            # ideal-gas mixture with condensates (Sec. 2, App. B)
TRACER_VAPOUR = 0
TRACER_CONDENSATE = 1


@dataclasses.dataclass
class Grid:
    """Structured grid, physical constants and hydrostatic reference profiles.

    ``rhobar_cell``/``pbar_cell`` have ``nz + 2G`` entries (ghost levels
    included, mirrored for a reflecting z boundary and wrapped for a periodic
    one); ``rhobar_face``/``pbar_face`` have ``nz + 1`` entries, index ``k``
    being the face between levels ``k-1`` and ``k``.
    """
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    gamma: float = 1.4
    grav: float = 9.81
    ntracer: int = 0
    bc: Tuple[int, int, int] = (BC_PERIODIC, BC_PERIODIC, BC_REFLECT)
    weno_eps: float = 1e-6
    weno_linear: bool = False
    rhobar_cell: Optional[np.ndarray] = None
    pbar_cell: Optional[np.ndarray] = None
    rhobar_face: Optional[np.ndarray] = None
    pbar_face: Optional[np.ndarray] = None
    # Mixture equation of state (used when eos == EOS_MIXTURE), per tracer:
    # kind (vapour or condensate); eps = molar mass / that of the dry gas
    # (vapours); sigma = heat capacity at constant volume / c_v of the dry
    # gas (c_ij / c_v,d for a condensate); mu = chemical potential (J/kg).
    eos: int = EOS_PASSIVE
    tracer_kind: Tuple[int, ...] = ()
    tracer_eps: Tuple[float, ...] = ()
    tracer_sigma: Tuple[float, ...] = ()
    tracer_mu: Tuple[float, ...] = ()
    # Sedimentation (mixture only): signed vertical velocity (m/s) of each
    # condensate relative to the air (negative: falling), and the dry gas
    # constant R_d (J/kg/K) that gives the temperature of the carried energy.
    tracer_wt: Tuple[float, ...] = ()
    rd: float = 0.0
    # Riemann solver at the faces: RIEMANN_LMARS (Sec. 4.1) or RIEMANN_HLLC
    riemann: int = 0

    @property
    def nvar(self) -> int:
        return 5 + self.ntracer

    @property
    def gy(self) -> int:
        return 0 if self.ny == 1 else G

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        """Padded state shape (nvar, nz+2G, ny+2Gy, nx+2G)."""
        return (self.nvar, self.nz + 2 * G, self.ny + 2 * self.gy, self.nx + 2 * G)

    @property
    def interior_shape(self) -> Tuple[int, int, int, int]:
        return (self.nvar, self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def interior(self, q):
        """View of the interior cells of a padded state array."""
        gy = self.gy
        return q[:, G:G + self.nz, gy:gy + self.ny, G:G + self.nx]

    def copy(self, **kw) -> "Grid":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Base states
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DryIsentropic:
    """Isentropic dry atmosphere: theta = theta0 everywhere, p = p0 at z = 0."""
    theta0: float = 300.0
    p0: float = 1.0e5
    rd: float = 287.0
    cp: float = 1004.5
    grav: float = 9.81

    def temperature(self, z):
        return self.theta0 - (self.grav / self.cp) * np.asarray(z, dtype=np.float64)

    def pressure(self, z):
        return self.p0 * (self.temperature(z) / self.theta0) ** (self.cp / self.rd)

    def density(self, z):
        return self.pressure(z) / (self.rd * self.temperature(z))

    def theta(self, z):
        return np.full_like(np.asarray(z, dtype=np.float64), self.theta0)


@dataclasses.dataclass
class AdiabatIsothermal:
    """Dry adiabat from (T0, p0) at z = 0 up to pressure p_top, isothermal above."""
    t0: float
    p0: float
    p_top: float
    rd: float
    cp: float
    grav: float

    @property
    def t_top(self) -> float:
        return self.t0 * (self.p_top / self.p0) ** (self.rd / self.cp)

    @property
    def z_top(self) -> float:
        return (self.t0 - self.t_top) * self.cp / self.grav

    def temperature(self, z):
        z = np.asarray(z, dtype=np.float64)
        return np.where(z < self.z_top, self.t0 - (self.grav / self.cp) * z, self.t_top)

    def pressure(self, z):
        z = np.asarray(z, dtype=np.float64)
        t = self.temperature(z)
        p_ad = self.p0 * (np.maximum(t, self.t_top) / self.t0) ** (self.cp / self.rd)
        h = self.rd * self.t_top / self.grav
        p_iso = self.p_top * np.exp(-(z - self.z_top) / h)
        return np.where(z < self.z_top, p_ad, p_iso)

    def density(self, z):
        return self.pressure(z) / (self.rd * self.temperature(z))

    def theta(self, z):
        return self.temperature(z) * (self.p0 / self.pressure(z)) ** (self.rd / self.cp)

    def z_of_pressure(self, p):
        """Height at which the base-state pressure equals ``p``."""
        if p >= self.p_top:
            t = self.t0 * (p / self.p0) ** (self.rd / self.cp)
            return (self.t0 - t) * self.cp / self.grav
        h = self.rd * self.t_top / self.grav
        return self.z_top + h * math.log(self.p_top / p)


def _pad_levels(interior: np.ndarray, bc_z: int) -> np.ndarray:
    """Extend a per-level profile by G ghost levels: mirrored or wrapped."""
    nz = interior.shape[0]
    out = np.empty(nz + 2 * G, dtype=np.float64)
    out[G:G + nz] = interior
    for m in range(G):
        if bc_z == BC_REFLECT:
            out[G - 1 - m] = interior[min(m, nz - 1)]
            out[G + nz + m] = interior[max(nz - 1 - m, 0)]
        else:
            out[G - 1 - m] = interior[(nz - 1 - m) % nz]
            out[G + nz + m] = interior[m % nz]
    return out


def reference_profiles(base, nz: int, dz: float, grav: float, bc_z: int = BC_REFLECT):
    """Hydrostatic reference profiles on the grid.

    Face pressure and density are the analytic base state at face heights,
    the cell pressure is the analytic value at the cell centre, and the cell
    density is defined by the discrete hydrostatic balance of the two
    bounding face pressures, (p_{k-1/2} - p_{k+1/2}) / (g dz), so that the
    perturbation form of the vertical momentum flux with the source
    -g (rho - rhobar_k) equals the full-pressure flux with the source
    -rho g (Sec. 2, momentum equation; Sec. 4.1, perturbation pressure).
    For g = 0 the cell density is the analytic value at the cell centre.
    """
    zf = np.arange(nz + 1, dtype=np.float64) * dz
    zc = (np.arange(nz, dtype=np.float64) + 0.5) * dz
    pf = base.pressure(zf)
    rf = base.density(zf)
    pc = base.pressure(zc)
    if grav != 0.0:
        rc = (pf[:-1] - pf[1:]) / (grav * dz)
    else:
        rc = base.density(zc)
    return _pad_levels(rc, bc_z), _pad_levels(pc, bc_z), rf.copy(), pf.copy()


def uniform_references(nz: int, rho0: float, p0: float):
    return (np.full(nz + 2 * G, rho0), np.full(nz + 2 * G, p0),
            np.full(nz + 1, rho0), np.full(nz + 1, p0))


# ---------------------------------------------------------------------------
# Initial conditions (host, FP64)
# ---------------------------------------------------------------------------

def state_from_primitives(grid: Grid, rho, u, v, w, p, tracers: Sequence = ()):
    """Padded conserved state from interior primitive fields of shape (nz, ny, nx).

    Ghost cells are left at zero: every library call fills them.
    """
    q = np.zeros(grid.shape, dtype=np.float64)
    qi = grid.interior(q)
    rho = np.broadcast_to(rho, (grid.nz, grid.ny, grid.nx))
    qi[0] = rho
    qi[1] = rho * u
    qi[2] = rho * v
    qi[3] = rho * w
    kin = 0.5 * rho * (np.asarray(u) ** 2 + np.asarray(v) ** 2 + np.asarray(w) ** 2)
    for t, qt in enumerate(tracers):
        qi[5 + t] = rho * qt
    if grid.eos == EOS_MIXTURE:
        qi[4] = mixture_internal_energy(grid, rho, p, [qi[5 + t] for t in range(grid.ntracer)]) + kin
        for t in range(grid.ntracer):
            qi[4] += grid.tracer_mu[t] * qi[5 + t]
    else:
        qi[4] = p / (grid.gamma - 1.0) + kin
    return q


def to_perturbation(grid: Grid, q):
    """The perturbation storage form of a padded state (numpy or torch, any
    float dtype): rho - rhobar_k in field 0 and E - pbar_k / (gamma - 1) in
    field 4 on every padded level k (the references' ghost levels included),
    the other fields unchanged. Returns a new array of q's type."""
    return _shift_storage(grid, q, -1.0)


def from_perturbation(grid: Grid, q):
    """The full conserved state from its perturbation storage form."""
    return _shift_storage(grid, q, 1.0)


def _shift_storage(grid: Grid, q, sign: float):
    rb = np.asarray(grid.rhobar_cell, dtype=np.float64)[:, None, None]
    eb = (np.asarray(grid.pbar_cell, dtype=np.float64) / (grid.gamma - 1.0))[:, None, None]
    if isinstance(q, np.ndarray):
        out = q.astype(np.float64, copy=True)
        out[0] += sign * rb
        out[4] += sign * eb
        return out.astype(q.dtype, copy=False)
    import torch

    out = q.clone()
    out[0] = out[0] + sign * torch.as_tensor(rb, dtype=q.dtype, device=q.device)
    out[4] = out[4] + sign * torch.as_tensor(eb, dtype=q.dtype, device=q.device)
    return out


def mixture_internal_energy(grid: Grid, rho, p, rho_t):
    """Internal energy per volume of a gas-condensate parcel at pressure p.

    From the species: the temperature follows from Dalton's law,
    p = R_d T (rho_d + sum over vapours rho_i / eps_i), and the internal
    energy is c_v,d T (rho_d + sum over all tracers sigma_t rho_t), with
    c_v,d = R_d / (gamma_d - 1) and rho_d = rho - sum rho_t.
    """
    rho_d = rho - sum(rho_t) if rho_t else rho
    gas = rho_d + sum(r / e for r, e, k in zip(rho_t, grid.tracer_eps, grid.tracer_kind)
                      if k == TRACER_VAPOUR)
    heat = rho_d + sum(r * s for r, s in zip(rho_t, grid.tracer_sigma))
    return p / (grid.gamma - 1.0) * heat / gas


def rest_fields(grid: Grid):
    """Hydrostatic rest: rho = cell reference density, p = cell reference pressure."""
    rc = grid.rhobar_cell[G:G + grid.nz][:, None, None]
    pc = grid.pbar_cell[G:G + grid.nz][:, None, None]
    shp = (grid.nz, grid.ny, grid.nx)
    return np.broadcast_to(rc, shp).copy(), np.broadcast_to(pc, shp).copy()


def theta_perturbed_density(rho_ref, theta_ref, dtheta):
    """Density after a potential-temperature perturbation at constant pressure.

    At fixed p, rho is inversely proportional to T and hence to theta
    (potential temperature, App. C).
    """
    return rho_ref * theta_ref / (theta_ref + dtheta)


def cell_centres(n: int, d: float):
    return (np.arange(n, dtype=np.float64) + 0.5) * d


def bubble_dtheta(grid: Grid, amp: float, radius: float, xc: float, zc: float, yc: Optional[float] = None):
    """Cosine-squared bubble: amp * cos^2(pi L / 2) for L = |x - xc| / radius <= 1."""
    x = cell_centres(grid.nx, grid.dx)[None, None, :]
    z = cell_centres(grid.nz, grid.dz)[:, None, None]
    r2 = (x - xc) ** 2 + (z - zc) ** 2
    if grid.ny > 1 and yc is not None:
        y = cell_centres(grid.ny, grid.dy)[None, :, None]
        r2 = r2 + (y - yc) ** 2
    L = np.sqrt(r2) / radius
    d = np.where(L <= 1.0, amp * np.cos(0.5 * np.pi * np.minimum(L, 1.0)) ** 2, 0.0)
    return np.broadcast_to(d, (grid.nz, grid.ny, grid.nx)).copy()


def dry_grid(nx, ny, nz, lx, ly, lz, bc=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT),
             base: Optional[DryIsentropic] = None, **kw) -> Tuple[Grid, DryIsentropic]:
    base = base or DryIsentropic()
    gamma = base.cp / (base.cp - base.rd)
    grid = Grid(nx=nx, ny=ny, nz=nz, dx=lx / nx, dy=ly / ny, dz=lz / nz,
                gamma=gamma, grav=base.grav, bc=tuple(bc), **kw)
    rc, pc, rf, pf = reference_profiles(base, nz, grid.dz, base.grav, bc[2])
    grid.rhobar_cell, grid.pbar_cell, grid.rhobar_face, grid.pbar_face = rc, pc, rf, pf
    return grid, base


def bubble_2d(nx=64, nz=64, lx=20e3, lz=10e3, amp=2.0, radius=2e3, zc=2e3, xc=None):
    """2-D dry rising bubble on an x-z grid (periodic x, reflecting z)."""
    grid, base = dry_grid(nx, 1, nz, lx, 1.0, lz, bc=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT))
    grid.dy = 1.0
    rho, p = rest_fields(grid)
    dth = bubble_dtheta(grid, amp, radius, lx / 2 if xc is None else xc, zc)
    rho = theta_perturbed_density(rho, base.theta0, dth)
    q = state_from_primitives(grid, rho, 0.0, 0.0, 0.0, p)
    return grid, q


def convection_3d(nx=256, ny=256, nz=128, lx=20e3, ly=20e3, lz=10e3, noise=0.1, nlev=10, seed=1):
    """3-D dry convection: seeded uniform theta noise in the lowest levels."""
    grid, base = dry_grid(nx, ny, nz, lx, ly, lz)
    rho, p = rest_fields(grid)
    rng = np.random.default_rng(seed)
    dth = np.zeros((nz, ny, nx))
    k = min(nlev, nz)
    dth[:k] = rng.uniform(-noise, noise, size=(k, ny, nx))
    rho = theta_perturbed_density(rho, base.theta0, dth)
    q = state_from_primitives(grid, rho, 0.0, 0.0, 0.0, p)
    return grid, q, dth


def convection_flow_3d(nx=256, ny=256, nz=128, lx=20e3, ly=20e3, lz=10e3, noise=0.1, nlev=10,
                       seed=1, flow_levels=16, seed_flow=37, p_amp=30.0):
    """Base point of the gradient workload: the convection state plus a seeded
    smooth flow in the top ``flow_levels`` levels.

    Returns (grid, base, dtheta, vel): the theta perturbation (K, shape
    (nz, ny, nx)) of ``convection_3d`` with the same seed, and a velocity
    field (m/s, shape (3, nz, ny, nx)) that is zero below the top levels.
    There each component is a sum of three horizontal Fourier modes with
    seeded wave numbers (1 to 3 per axis), phases and weights, scaled by a
    vertical envelope sin^2 that rises from about 0 at the lowest flow level
    to 1 at the top: u = e (3 + 1.5 m_u), v = e (2 + 1 m_v) and w = e m_w,
    with |m| <= 1. The horizontal components are then positive, so no x or y
    interface velocity crosses zero where the upwind side of the Riemann flux
    switches, and the flow is smooth, so that where the vertical one does the
    two sides' states nearly agree and the switch leaves the map almost
    differentiable. Without the flow the top levels are at rest for the whole
    run (sound crosses about 60 levels in 200 steps) and a kinetic-energy loss
    there is quadratic in round-off velocities.

    Also returned: a smooth pressure perturbation dp (Pa, (nz, ny, nx)) of
    amplitude ``p_amp`` everywhere, three seeded horizontal modes times
    cos(pi kz z / lz) (kz in {1, 2}, so it mirrors smoothly at the lids).
    Without it p - pbar is round-off, and any perturbation of the state moves
    it across sqrt(weno_eps) (about 1e-3 Pa), the scale on which the
    Jiang-Shu weights of p' bend; with it p' varies by Pa from cell to cell
    and small perturbations stay in the weights' smooth regime. The state
    follows from these by ``state_from_theta``.
    """
    grid, base = dry_grid(nx, ny, nz, lx, ly, lz)
    rng = np.random.default_rng(seed)
    dth = np.zeros((nz, ny, nx))
    k = min(nlev, nz)
    dth[:k] = rng.uniform(-noise, noise, size=(k, ny, nx))
    vel = np.zeros((3, nz, ny, nx))
    kf = min(flow_levels, nz)
    fr = np.random.default_rng(seed_flow)
    x = cell_centres(nx, 1.0 / nx)[None, :]
    y = cell_centres(ny, 1.0 / ny)[:, None]

    def modes():
        m = np.zeros((ny, nx))
        wts = fr.uniform(0.5, 1.0, size=3)
        for a in wts:
            kx, ky = fr.integers(1, 4, size=2)
            ph = fr.uniform(0.0, 2.0 * np.pi)
            m += a * np.sin(2.0 * np.pi * (kx * x + ky * y) + ph)
        return m / wts.sum()

    mu, mv, mw = modes(), modes(), modes()
    lev = np.arange(kf, dtype=np.float64)
    env = np.sin(0.5 * np.pi * (lev + 0.5) / kf) ** 2
    for j, (c, a, m) in enumerate(((3.0, 1.5, mu), (2.0, 1.0, mv), (0.0, 1.0, mw))):
        vel[j, nz - kf:] = env[:, None, None] * (c + a * m)[None]
    zc = cell_centres(nz, 1.0 / nz)[:, None, None]
    dp = np.zeros((nz, ny, nx))
    pw = fr.uniform(0.5, 1.0, size=3)
    for a in pw:
        kz = fr.integers(1, 3)
        dp += a * np.cos(np.pi * kz * zc) * modes()[None]
    dp *= p_amp / pw.sum()
    return grid, base, dth, vel, dp


def state_from_theta(grid: Grid, base: DryIsentropic, dtheta, vel, dp=None):
    """Padded conserved state (torch) from a theta perturbation and a velocity field.

    The density is perturbed at constant pressure, rho = rhobar_k theta0 /
    (theta0 + theta'), the pressure is the cell reference pbar_k plus ``dp``
    (if given), and E = p / (gamma - 1) + rho |u|^2 / 2; ghost cells are zero.
    ``dtheta`` (nz, ny, nx), ``vel`` (3, nz, ny, nx) and ``dp`` are torch
    tensors of one dtype and device; the result has that dtype and device and
    is differentiable in them (torch autograd), so that a gradient with
    respect to the state's interior carries over to one with respect to
    theta'.
    """
    import torch

    dev, dt_ = dtheta.device, dtheta.dtype
    nz = grid.nz
    rc = torch.as_tensor(grid.rhobar_cell[G:G + nz], dtype=dt_, device=dev)[:, None, None]
    pc = torch.as_tensor(grid.pbar_cell[G:G + nz], dtype=dt_, device=dev)[:, None, None]
    rho = rc * base.theta0 / (base.theta0 + dtheta)
    mom = rho * vel
    p = pc if dp is None else pc + dp
    e = p / (grid.gamma - 1.0) + 0.5 * rho * (vel * vel).sum(dim=0)
    q = torch.zeros(grid.shape, dtype=dt_, device=dev)
    gy = grid.gy
    inner = q[:, G:G + nz, gy:gy + grid.ny, G:G + grid.nx]
    inner[0] = rho
    inner[1:4] = mom
    inner[4] = e
    return q


JOVIAN_MU = 2.3e-3       # kg/mol
JOVIAN_CP = 12400.0      # J/(kg K)
JOVIAN_G = 24.79         # m/s^2


def jovian_base() -> AdiabatIsothermal:
    rd = RGAS / JOVIAN_MU
    return AdiabatIsothermal(t0=800.0, p0=200e5, p_top=0.2e5, rd=rd, cp=JOVIAN_CP, grav=JOVIAN_G)


def jovian_3d(nx=512, ny=512, nz=256, dxy=5.5e3, lz=400e3, seed_q=2, seed_theta=3,
              condense_p=(7e5, 0.7e5), noise=0.1, nlev=10, mixture=False):
    """3-D Jovian-like column: H2-He gas, two vapours and two (zero) clouds,
    passive or (``mixture``) under the mixture equation of state with the
    water / ammonia table of ``condensable_species``."""
    base = jovian_base()
    gamma = base.cp / (base.cp - base.rd)
    grid = Grid(nx=nx, ny=ny, nz=nz, dx=dxy, dy=dxy, dz=lz / nz, gamma=gamma,
                grav=base.grav, ntracer=4, bc=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT))
    if mixture:
        grid = with_mixture(grid, condensable_species(base.cp - base.rd, JOVIAN_MU))
    rc, pc, rf, pf = reference_profiles(base, nz, grid.dz, base.grav, BC_REFLECT)
    grid.rhobar_cell, grid.pbar_cell, grid.rhobar_face, grid.pbar_face = rc, pc, rf, pf
    rho, p = rest_fields(grid)
    zc = cell_centres(nz, grid.dz)
    rng = np.random.default_rng(seed_q)
    tr = []
    for pc_ in condense_p:
        zcond = base.z_of_pressure(pc_)
        qv = 10.0 ** rng.uniform(-4.0, -2.0, size=(nz, ny, nx))
        qv[zc >= zcond] = 0.0
        tr.append(qv)
    tr.append(np.zeros((nz, ny, nx)))
    tr.append(np.zeros((nz, ny, nx)))
    rng_t = np.random.default_rng(seed_theta)
    dth = np.zeros((nz, ny, nx))
    k = min(nlev, nz)
    dth[:k] = rng_t.uniform(-noise, noise, size=(k, ny, nx))
    th = base.theta(zc)[:, None, None]
    rho = theta_perturbed_density(rho, th, dth)
    q = state_from_primitives(grid, rho, 0.0, 0.0, 0.0, p, tr)
    return grid, q


# Condensables: molar mass (kg/mol), c_v and c_p of the vapour, heat capacity
# of the condensate (J/kg/K), latent heat (J/kg) and saturation vapour
# pressure (Pa) at the reference (triple-point) temperature (K); textbook values.
WATER = dict(molar=18.015e-3, cv_vap=1385.0, cp_vap=1847.0, c_cond=4184.0, latent=2.501e6,
             t_ref=273.16, p_ref=611.7)
AMMONIA = dict(molar=17.031e-3, cv_vap=1572.0, cp_vap=2060.0, c_cond=4700.0, latent=1.371e6,
               t_ref=195.4, p_ref=6060.0)


def _vapour(sp, cvd, mu_dry):
    return (TRACER_VAPOUR, sp["molar"] / mu_dry, sp["cv_vap"] / cvd, 0.0)


def _condensate(sp, cvd):
    # chemical potential of the condensate: -(L^r + (c_cond - c_p,vap) T^r) (Sec. 2, eq. muij)
    mu = -(sp["latent"] + (sp["c_cond"] - sp["cp_vap"]) * sp["t_ref"])
    return (TRACER_CONDENSATE, 1.0, sp["c_cond"] / cvd, mu)


def condensable_species(cvd: float, mu_dry: float):
    """Water and ammonia vapours and their clouds, as mixture-equation-of-state
    tracers of a gas with c_v = ``cvd`` (J/kg/K) and molar mass ``mu_dry``
    (kg/mol): (kind, molar-mass ratio, heat capacity over cvd, chemical
    potential). Vapour potentials are zero."""
    return (_vapour(WATER, cvd, mu_dry), _vapour(AMMONIA, cvd, mu_dry),
            _condensate(WATER, cvd), _condensate(AMMONIA, cvd))


def kessler_tracers(cvd: float, mu_dry: float, rd: float, species=(WATER, AMMONIA),
                    k=(0.3, 1e-3, 2.2, 0.5)):
    """Tracer table [vapours, clouds, precipitations] of ``species`` and the
    Kessler parameters (rate coefficients k = (k1, k2, k3, k4); saturation
    vapour pressure from the species' latent heat and heat capacities)."""
    n = len(species)
    table = ([_vapour(sp, cvd, mu_dry) for sp in species] + [_condensate(sp, cvd) for sp in species]
             + [_condensate(sp, cvd) for sp in species])
    kes = []
    for i, sp in enumerate(species):
        beta, delta = clausius_clapeyron(sp["latent"], sp["c_cond"] - sp["cp_vap"],
                                         RGAS / sp["molar"], sp["t_ref"])
        kes.append(KesslerSpecies(vapour=i, cloud=n + i, precip=2 * n + i, k1=k[0], k2=k[1], k3=k[2],
                                  k4=k[3], p_ref=sp["p_ref"], t_ref=sp["t_ref"], beta=beta,
                                  delta=delta, eps=sp["molar"] / mu_dry))
    return tuple(table), Kessler(species=tuple(kes), rd=rd)


def with_mixture(grid: Grid, species) -> Grid:
    """The grid with the mixture equation of state and these tracers."""
    return grid.copy(eos=EOS_MIXTURE, ntracer=len(species),
                     tracer_kind=tuple(int(s[0]) for s in species),
                     tracer_eps=tuple(float(s[1]) for s in species),
                     tracer_sigma=tuple(float(s[2]) for s in species),
                     tracer_mu=tuple(float(s[3]) for s in species))


@dataclasses.dataclass
class KesslerSpecies:
    """One condensable of the Kessler scheme (Sec. 3), as parameters.

    vapour, cloud, precip: tracer indices of its vapour, cloud and
    precipitation (mixture equation of state: one vapour, two condensates);
    k1 condensation (1/s), k2 autoconversion (1/s), k3 accretion and k4
    evaporation (1/s per unit mixing ratio); saturation vapour pressure over
    the cloud p* = p_ref exp[beta (1 - 1/t) - delta ln t] with t = T / t_ref
    (App. D); eps: molar mass over that of the dry gas.
    """
    vapour: int
    cloud: int
    precip: int
    k1: float
    k2: float
    k3: float
    k4: float
    p_ref: float
    t_ref: float
    beta: float
    delta: float
    eps: float


@dataclasses.dataclass
class Kessler:
    """Kessler microphysics of a grid: its condensables, the dry gas constant,
    and the stopping rule of the Newton iteration (step size below
    ``tol`` times the species' total mixing ratio, at most ``max_iter``)."""
    species: Tuple[KesslerSpecies, ...]
    rd: float
    max_iter: int = 30
    tol: float = 1e-14


@dataclasses.dataclass(frozen=True)
class SatAdjSpecies:
    """One vapour / cloud pair of the saturation adjustment (App. D): tracer
    indices of the vapour and of its cloud, and the saturation vapour pressure
    over the cloud p* = p_ref exp[beta (1 - 1/t) - delta ln t], t = T / t_ref."""
    vapour: int
    cloud: int
    p_ref: float
    t_ref: float
    beta: float
    delta: float


@dataclasses.dataclass(frozen=True)
class SatAdjust:
    """Saturation adjustment of a grid: its vapour / cloud pairs, the dry gas
    constant, and the stopping rule (a transfer below ``tol`` times the pair's
    total density, at most ``max_iter`` sweeps over the pairs)."""
    species: Tuple[SatAdjSpecies, ...]
    rd: float
    max_iter: int = 20
    tol: float = 1e-14


def saturation_tracers(cvd: float, mu_dry: float, rd: float, species=(WATER, AMMONIA)):
    """Tracer table [vapours, clouds] of ``species`` and their saturation
    adjustment parameters."""
    n = len(species)
    table = [_vapour(sp, cvd, mu_dry) for sp in species] + [_condensate(sp, cvd) for sp in species]
    pairs = []
    for i, sp in enumerate(species):
        beta, delta = clausius_clapeyron(sp["latent"], sp["c_cond"] - sp["cp_vap"],
                                         RGAS / sp["molar"], sp["t_ref"])
        pairs.append(SatAdjSpecies(vapour=i, cloud=n + i, p_ref=sp["p_ref"], t_ref=sp["t_ref"],
                                   beta=beta, delta=delta))
    return tuple(table), SatAdjust(species=tuple(pairs), rd=rd)


def clausius_clapeyron(latent_ref: float, dc: float, r_vap: float, t_ref: float):
    """(beta, delta) of App. D from the latent heat at t_ref, c_cond - c_p,vap and R_vap."""
    return (latent_ref + dc * t_ref) / (r_vap * t_ref), dc / r_vap


def jovian_kessler_3d(nx=512, ny=512, nz=256, seed_q=2, seed_theta=3, sediment=False, **kw):
    """The Jovian-like column with water and ammonia vapour, cloud and
    precipitation under the mixture equation of state, and the Kessler
    parameters of the two species: (grid, state, Kessler); ``sediment``: the
    precipitation falls."""
    base = jovian_base()
    grid, q = jovian_3d(nx=nx, ny=ny, nz=nz, seed_q=seed_q, seed_theta=seed_theta, **kw)
    table, kes = kessler_tracers(base.cp - base.rd, JOVIAN_MU, base.rd)
    g6 = with_mixture(grid, table)
    rho = grid.interior(q)[0]
    p = rest_fields(grid)[1]
    shp = rho.shape
    zc = cell_centres(nz, grid.dz)[:, None, None]
    rng = np.random.default_rng(seed_q + 100)
    vap = []
    for pc_ in (7e5, 0.7e5):   # up to 20 km above the condensation level: supersaturated there
        qv = 10.0 ** rng.uniform(-3.0, -0.9, size=shp)
        vap.append(np.where(zc < base.z_of_pressure(pc_) + 20e3, qv, 0.0))
    seeds = [10.0 ** rng.uniform(-6.0, -4.0, size=shp) for _ in range(4)]
    if sediment:   # water and ammonia rain fall at 8 and 5 m/s
        g6 = g6.copy(tracer_wt=(0.0, 0.0, 0.0, 0.0, -8.0, -5.0), rd=base.rd)
    q6 = state_from_primitives(g6, rho, 0.0, 0.0, 0.0, p, vap + seeds)
    return g6, q6, kes


def jovian_satadj_3d(nx=512, ny=512, nz=256, seed_q=2, seed_theta=3, **kw):
    """The Jovian-like column with water and ammonia vapour and cloud under
    the mixture equation of state (4 tracers), vapour supersaturated up to
    20 km above each condensation level and clouds seeded, and the saturation
    adjustment parameters of the two species: (grid, state, SatAdjust)."""
    base = jovian_base()
    grid, q = jovian_3d(nx=nx, ny=ny, nz=nz, seed_q=seed_q, seed_theta=seed_theta, **kw)
    table, adj = saturation_tracers(base.cp - base.rd, JOVIAN_MU, base.rd)
    g4 = with_mixture(grid, table)
    rho = grid.interior(q)[0]
    p = rest_fields(grid)[1]
    shp = rho.shape
    zc = cell_centres(nz, grid.dz)[:, None, None]
    rng = np.random.default_rng(seed_q + 200)
    vap = []
    for pc_ in (7e5, 0.7e5):
        qv = 10.0 ** rng.uniform(-3.0, -0.9, size=shp)
        vap.append(np.where(zc < base.z_of_pressure(pc_) + 20e3, qv, 0.0))
    clouds = [10.0 ** rng.uniform(-6.0, -4.0, size=shp) for _ in range(2)]
    q4 = state_from_primitives(g4, rho, 0.0, 0.0, 0.0, p, vap + clouds)
    return g4, q4, adj


ENSEMBLE_SIZES = ((128, 128), (256, 128), (384, 192), (512, 256))


def ensemble_2d(n=64, seed=4, lx=20e3, lz=10e3, sizes=ENSEMBLE_SIZES):
    """Ensemble of 2-D bubbles with seeded sizes, amplitudes and radii."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(sizes), size=n)
    amps = rng.uniform(0.5, 3.0, size=n)
    radii = rng.uniform(1e3, 3e3, size=n)
    members = []
    for m in range(n):
        nx, nz = sizes[idx[m]]
        members.append(bubble_2d(nx=nx, nz=nz, lx=lx, lz=lz, amp=float(amps[m]), radius=float(radii[m])))
    return members


def random_smooth_state(grid: Grid, seed: int, amp_rho=0.02, amp_u=5.0, amp_p=50.0, amp_q=1e-3):
    """Seeded smooth-plus-noise perturbation of hydrostatic rest, all fields active.

    Used for parity cases where every term of the right-hand side is nonzero.
    """
    rng = np.random.default_rng(seed)
    rho, p = rest_fields(grid)
    shp = (grid.nz, grid.ny, grid.nx)
    x = cell_centres(grid.nx, 1.0 / grid.nx)[None, None, :]
    y = cell_centres(grid.ny, 1.0 / grid.ny)[None, :, None]
    z = cell_centres(grid.nz, 1.0 / grid.nz)[:, None, None]

    def field(scale):
        ph = rng.uniform(0, 2 * np.pi, size=3)
        smooth = np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * y + ph[1]) * np.sin(np.pi * z + ph[2])
        return scale * (np.broadcast_to(smooth, shp) + 0.3 * rng.standard_normal(shp))

    rho = rho * (1.0 + field(amp_rho))
    u = field(amp_u)
    v = field(amp_u) if grid.ny > 1 else np.zeros(shp)
    w = field(amp_u)
    p = p + field(amp_p)
    trs = [np.abs(field(amp_q)) + amp_q for _ in range(grid.ntracer)]
    return state_from_primitives(grid, rho, u, v, w, p, trs)


def seeded_normal(shape, seed: int):
    return np.random.default_rng(seed).standard_normal(shape)
