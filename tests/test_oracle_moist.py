"""Pins of the oracle's mixture equation of state (Sec. 2, eqs. energy, eos and
tv; App. B, eq. p2 and the effective adiabatic index).

The pins come from the physics of the mixture, not from the formula the
oracle evaluates: states are built species by species from a temperature
(Dalton's law for the pressure, summed heat capacities for the internal
energy, chemical energy per unit mass), the frozen sound speed follows from
the mixture's gas constant and heat capacity, and exact reductions (passive
tracers, a uniform mixture as one ideal gas, the chemical-potential term as
an advected quantity) must hold to rounding.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O

RD = 3614.98          # J/(kg K), an H2-He gas
GAMMA_D = 1.41149
CVD = RD / (GAMMA_D - 1.0)
# two vapours and their condensates: kind, eps (molar-mass ratio), sigma (heat capacity / c_v,d), mu (J/kg)
SPECIES = (
    (W.TRACER_VAPOUR, 18.0 / 2.3, 1385.0 / CVD, 0.0),
    (W.TRACER_VAPOUR, 17.0 / 2.3, 1572.0 / CVD, 0.0),
    (W.TRACER_CONDENSATE, 1.0, 4184.0 / CVD, -3.14e6),
    (W.TRACER_CONDENSATE, 1.0, 4700.0 / CVD, -1.9e6),
)


def mixture_grid(nx, ny, nz, bc=(0, 0, 0), grav=0.0, species=SPECIES, eos=W.EOS_MIXTURE):
    g = W.Grid(nx=nx, ny=ny, nz=nz, dx=100.0, dy=120.0, dz=90.0, gamma=GAMMA_D, grav=grav, bc=bc,
               ntracer=len(species), eos=eos,
               tracer_kind=tuple(s[0] for s in species), tracer_eps=tuple(s[1] for s in species),
               tracer_sigma=tuple(s[2] for s in species), tracer_mu=tuple(s[3] for s in species))
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(nz, 0.5, 2.0e5)
    return g


def species_state(g, rho_d, rho_t, T, u, v, w, species=SPECIES):
    """Padded conserved state from species densities and temperature.

    p = R_d T (rho_d + sum_vapour rho_i / eps_i)                (Dalton)
    E = c_v,d T (rho_d + sum_t sigma_t rho_t) + K + sum mu_t rho_t
    """
    rho = rho_d + sum(rho_t)
    p = RD * T * (rho_d + sum(r / s[1] for r, s in zip(rho_t, species) if s[0] == W.TRACER_VAPOUR))
    E = (CVD * T * (rho_d + sum(s[2] * r for r, s in zip(rho_t, species)))
         + 0.5 * rho * (u * u + v * v + w * w) + sum(s[3] * r for r, s in zip(rho_t, species)))
    q = np.zeros(g.shape)
    qi = g.interior(q)
    qi[0], qi[1], qi[2], qi[3], qi[4] = rho, rho * u, rho * v, rho * w, E
    for t, r in enumerate(rho_t):
        qi[5 + t] = r
    return q, p, rho


def random_species(g, seed):
    rng = np.random.default_rng(seed)
    shp = (g.nz, g.ny, g.nx)
    rho_d = 0.5 * (1.0 + 0.1 * rng.standard_normal(shp))
    rho_t = [rho_d * 10.0 ** rng.uniform(-4.0, -1.5, size=shp) for _ in SPECIES]
    T = 300.0 * (1.0 + 0.05 * rng.standard_normal(shp))
    u, v, w = (8.0 * rng.standard_normal(shp) for _ in range(3))
    return rho_d, rho_t, T, u, v, w


def frozen_gamma(rho_d, rho_t):
    """c_p / c_v of the parcel: 1 + (rho R)_mix / (rho c_v)_mix (condensates carry heat, no pressure)."""
    rR = RD * (rho_d + sum(r / s[1] for r, s in zip(rho_t, SPECIES) if s[0] == W.TRACER_VAPOUR))
    rc = CVD * (rho_d + sum(s[2] * r for r, s in zip(rho_t, SPECIES)))
    return 1.0 + rR / rc


def test_mixture_pressure_is_daltons_law():
    g = mixture_grid(7, 5, 6)
    rho_d, rho_t, T, u, v, w = random_species(g, 1)
    q, p_true, _ = species_state(g, rho_d, rho_t, T, u, v, w)
    prim = O.cons_to_prim(torch.as_tensor(q), g)
    p = g.interior(prim["p"].unsqueeze(0).numpy())[0]
    assert np.max(np.abs(p / p_true - 1.0)) < 1e-13


def test_mixture_sound_speed_is_the_frozen_one():
    g = mixture_grid(6, 4, 5)
    rho_d, rho_t, T, u, v, w = random_species(g, 2)
    q, p, rho = species_state(g, rho_d, rho_t, T, u, v, w)
    c = np.sqrt(frozen_gamma(rho_d, rho_t) * p / rho)
    s = (np.abs(u) + c) / g.dx + (np.abs(v) + c) / g.dy + (np.abs(w) + c) / g.dz
    dt = O.cfl_dt(q, g, 0.9)
    assert abs(dt - 0.9 / s.max()) <= 1e-13 * dt


def test_uniform_mixture_is_one_ideal_gas():
    """With the same mass fractions everywhere and no chemical energy, the
    mixture is one ideal gas with the frozen gamma: its right-hand side equals
    the passive one with that gamma."""
    species = tuple((k, e, s, 0.0) for k, e, s, _ in SPECIES)
    g = mixture_grid(10, 8, 9, bc=(0, 0, 1), grav=9.0, species=species)
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.reference_profiles(
        W.DryIsentropic(), 9, g.dz, 9.0, 1)
    fr = np.array([3e-3, 2e-3, 1e-3, 5e-4])        # mass fractions
    rho0, _, _, _, _, _ = random_species(g, 3)
    rho = rho0 / 0.5 * g.rhobar_cell[3:-3][:, None, None]
    rho_t = [f * rho for f in fr]
    rho_d = rho - sum(rho_t)
    gam = float(frozen_gamma(np.ones(1) * (1.0 - fr.sum()), [np.ones(1) * f for f in fr])[0])
    rng = np.random.default_rng(4)
    shp = rho.shape
    u, v, w = (5.0 * rng.standard_normal(shp) for _ in range(3))
    p = g.pbar_cell[3:-3][:, None, None] * (1.0 + 1e-3 * rng.standard_normal(shp))
    gp = g.copy(eos=W.EOS_PASSIVE, gamma=gam)
    q = W.state_from_primitives(gp, rho, u, v, w, p, [f * np.ones(shp) for f in fr])
    r_mix = O.rhs(q, g).numpy()
    r_one = O.rhs(q, gp).numpy()
    for m in range(g.nvar):
        scale = np.max(np.abs(r_one[m]))
        assert np.max(np.abs(r_mix[m] - r_one[m])) <= 1e-11 * scale, m
    # and the state built from species at the same T has the same pressure
    T = p / (RD * (rho_d + sum(r / s[1] for r, s in zip(rho_t, species) if s[0] == W.TRACER_VAPOUR)))
    qs, p_true, _ = species_state(g, rho_d, rho_t, T, u, v, w, species)
    assert np.max(np.abs(g.interior(qs)[4] / g.interior(q)[4] - 1.0)) < 1e-13


def test_chemical_energy_is_advected_with_its_tracer():
    """Adding sum mu_t rho_t to E and switching the chemical potentials on
    leaves the pressure unchanged and adds sum mu_t R[rho_t] to R[E]."""
    g1 = mixture_grid(9, 7, 8, bc=(0, 0, 1), grav=9.0)
    g0 = g1.copy(tracer_mu=(0.0,) * 4)
    rho_d, rho_t, T, u, v, w = random_species(g1, 5)
    q1, _, _ = species_state(g1, rho_d, rho_t, T, u, v, w)
    q0 = q1.copy()
    chem = sum(s[3] * r for r, s in zip(rho_t, SPECIES))
    g0.interior(q0)[4] -= chem
    r0 = O.rhs(q0, g0).numpy()
    r1 = O.rhs(q1, g1).numpy()
    for m in range(g1.nvar):
        expect = r0[m] + (sum(s[3] * r0[5 + t] for t, s in enumerate(SPECIES)) if m == 4 else 0.0)
        scale = max(np.max(np.abs(r1[m])), np.max(np.abs(expect)))
        assert np.max(np.abs(r1[m] - expect)) <= 1e-10 * scale, m


def test_passive_reduction():
    """Vapours whose heat-capacity ratio is 1/eps, no condensates, no chemical
    energy: the mixture right-hand side is the passive one."""
    species = ((W.TRACER_VAPOUR, 18.0 / 2.3, 2.3 / 18.0, 0.0), (W.TRACER_VAPOUR, 17.0 / 2.3, 2.3 / 17.0, 0.0))
    g = mixture_grid(8, 6, 7, bc=(0, 1, 1), species=species)
    q = W.random_smooth_state(g.copy(eos=W.EOS_PASSIVE), seed=6)
    r_mix = O.rhs(q, g).numpy()
    r_pas = O.rhs(q, g.copy(eos=W.EOS_PASSIVE)).numpy()
    for m in range(g.nvar):
        assert np.max(np.abs(r_mix[m] - r_pas[m])) <= 1e-13 * np.max(np.abs(r_pas[m])), m


def test_mixture_free_stream_is_exact():
    g = mixture_grid(10, 6, 8, bc=(0, 0, 0))
    shp = (g.nz, g.ny, g.nx)
    rho_d = np.full(shp, 0.45)
    rho_t = [np.full(shp, 0.45 * f) for f in (3e-3, 2e-3, 1e-3, 5e-4)]
    q, _, _ = species_state(g, rho_d, rho_t, np.full(shp, 280.0), 4.0, -3.0, 2.0)
    assert float(O.rhs(q, g).abs().max()) == 0.0


def test_mixture_conserves_mass_tracers_and_energy():
    g = mixture_grid(12, 10, 8, bc=(0, 0, 0))
    rho_d, rho_t, T, u, v, w = random_species(g, 7)
    q, _, _ = species_state(g, rho_d, rho_t, T, u, v, w)
    s0 = O.conservation_sums(q, g)
    dt = O.cfl_dt(q, g, 0.9)
    qn = O.run(q, g, dt, 5)
    s1 = O.conservation_sums(qn, g)
    scale = np.abs(g.interior(q)).reshape(g.nvar, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale
