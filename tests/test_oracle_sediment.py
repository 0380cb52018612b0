"""Pins of the oracle's sedimentation of condensates (Sec. 2: eq. d3, the
momentum equations and the total-energy equation with the terminal velocity).

* a uniform state is left alone by the sedimentation fluxes, and with gravity
  the energy gains exactly the frictional heating -g rho_t w_t;
* in a periodic column mass, momentum and energy are conserved;
* in a column with walls, at hydrostatic rest, the condensate mass and the
  energy change only by what leaves through the ground, w_t rho_t and
  w_t rho_t e_t of the lowest cell, with e_t = c_t T + mu_t built here from the
  species (Dalton's law for T), and by the heating source;
* no condensate enters through the lid.
"""
import numpy as np
import torch

import workloads as W
from oracle import snap_oracle as O

RD, GD = 287.0, 1.4
CVD = RD / (GD - 1.0)
EPS = 18.015e-3 / (W.RGAS / RD)
SPECIES = ((W.TRACER_VAPOUR, EPS, 1385.0 / CVD, 0.0),
           (W.TRACER_CONDENSATE, 1.0, 4184.0 / CVD, -3.14e6),      # cloud, no fall speed
           (W.TRACER_CONDENSATE, 1.0, 4184.0 / CVD, -3.14e6))      # rain
WT = (0.0, 0.0, -6.0)


def grid(nx, ny, nz, bc, grav, base=None, wt=WT):
    if base is None:
        g = W.Grid(nx=nx, ny=ny, nz=nz, dx=100.0, dy=100.0, dz=50.0, gamma=GD, grav=grav, bc=bc)
        g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(nz, 1.1, 9e4)
    else:
        g, _ = W.dry_grid(nx, ny, nz, 100.0 * nx, 100.0 * ny, 50.0 * nz, bc=bc, base=base)
    g = W.with_mixture(g, SPECIES)
    return g.copy(tracer_wt=tuple(wt), rd=RD)


def uniform_state(g):
    shp = (g.nz, g.ny, g.nx)
    return W.state_from_primitives(g, np.full(shp, 1.1), 0.0, 0.0, 0.0, 9e4,
                                   [np.full(shp, 8e-3), np.full(shp, 1e-3), np.full(shp, 2e-3)])


def test_uniform_state_only_heats():
    g0 = grid(6, 5, 8, (0, 0, 0), 0.0)
    q = uniform_state(g0)
    assert float(O.rhs(q, g0).abs().max()) == 0.0
    g = grid(6, 5, 8, (0, 0, 0), 9.81)
    r = O.rhs(q, g).numpy()
    rain = g.interior(q)[7]
    assert np.allclose(r[4], -9.81 * WT[2] * rain, rtol=1e-14, atol=0)
    r_dry = O.rhs(q, g.copy(tracer_wt=(0.0, 0.0, 0.0))).numpy()
    assert np.array_equal(np.delete(r, 4, axis=0), np.delete(r_dry, 4, axis=0))


def test_periodic_column_conserves():
    g = grid(6, 5, 12, (0, 0, 0), 0.0)
    q = W.random_smooth_state(g, seed=3, amp_q=2e-3)
    r = O.rhs(q, g).numpy()
    for m in range(g.nvar):
        scale = np.max(np.abs(r[m])) * r[m].size
        assert abs(r[m].sum()) <= 1e-13 * scale, m


def _rest_column(nz, wt=WT):
    g = grid(3, 2, nz, (0, 0, 1), 9.81, base=W.DryIsentropic(), wt=wt)
    rho, p = W.rest_fields(g)
    rng = np.random.default_rng(5)
    shp = rho.shape
    qv = 5e-3 * np.ones(shp)
    qc = 10.0 ** rng.uniform(-5, -3, shp)
    qr = 10.0 ** rng.uniform(-5, -3, shp)
    return g, W.state_from_primitives(g, rho, 0.0, 0.0, 0.0, p, [qv, qc, qr]), (rho, p, qv, qc, qr)


def test_wall_column_loses_rain_only_through_the_ground():
    g, q, (rho, p, qv, qc, qr) = _rest_column(16)
    r = O.rhs(q, g).numpy()
    r_off = O.rhs(q, g.copy(tracer_wt=(0.0, 0.0, 0.0))).numpy()
    sed = r - r_off
    rain = g.interior(q)[7]
    # mass: d/dt sum(rho_r dz) = w_t rho_r(ground); the lid lets nothing in
    lost = WT[2] * rain[0]
    assert np.allclose(sed[7].sum(axis=0) * g.dz, lost, rtol=1e-12, atol=0)
    assert np.allclose(sed[0].sum(axis=0) * g.dz, lost, rtol=1e-12, atol=0)
    # energy: what leaves carries e_t = c_t T + mu_t (at rest), plus the heating
    gas = (1.0 - qv - qc - qr) + qv / EPS                     # Dalton, per unit mass
    T = p / (RD * rho * gas)
    e_rain = SPECIES[2][2] * CVD * T + SPECIES[2][3]
    heat = -9.81 * WT[2] * rain
    expect = WT[2] * rain[0] * e_rain[0] + (heat * g.dz).sum(axis=0)
    assert np.allclose(sed[4].sum(axis=0) * g.dz, expect, rtol=1e-11, atol=0)
    # cloud and vapour do not fall
    assert np.array_equal(sed[5], np.zeros_like(sed[5])) and np.array_equal(sed[6], np.zeros_like(sed[6]))


def test_rising_condensate_leaves_through_the_lid():
    g, q, _ = _rest_column(10, wt=(0.0, 0.0, 4.0))
    sed = (O.rhs(q, g) - O.rhs(q, g.copy(tracer_wt=(0.0, 0.0, 0.0)))).numpy()
    rain = g.interior(q)[7]
    assert np.allclose(sed[7].sum(axis=0) * g.dz, -4.0 * rain[-1], rtol=1e-12, atol=0)


def test_rain_falls_into_the_cell_below():
    g, q, _ = _rest_column(12)
    qi = g.interior(q)
    qi[7] = 0.0
    qi[7, 6] = 1e-3 * qi[0, 6]          # rain in level 6 only
    sed = (O.rhs(q, g) - O.rhs(q, g.copy(tracer_wt=(0.0, 0.0, 0.0)))).numpy()[7]
    assert np.all(sed[6] < 0) and np.all(sed[5] > 0)
    assert np.allclose(sed[5], -sed[6], rtol=1e-14, atol=0)
    others = np.delete(sed, [5, 6], axis=0)
    assert np.all(others == 0.0)
