"""Pins of the whole oracle right-hand side and step against invariants the
method fixes: free stream, hydrostatic rest, conservation, tracer
consistency and mirror symmetry."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O


def _uniform_grid(nx, ny, nz, bc, ntracer=0):
    g = W.Grid(nx=nx, ny=ny, nz=nz, dx=10.0, dy=12.0, dz=9.0, grav=0.0, bc=bc, ntracer=ntracer)
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(nz, 1.1, 1.0e5)
    return g


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 0, 1), (1, 1, 1)])
def test_free_stream_is_exact(bc):
    g = _uniform_grid(12, 8, 10, bc, ntracer=2)
    vel = [3.0, -2.0, 1.5]
    for a in range(3):
        if bc[a] == 1:
            vel[a] = 0.0        # no flow through a wall
    shp = (g.nz, g.ny, g.nx)
    q = W.state_from_primitives(g, np.full(shp, 1.2), vel[0], vel[1], vel[2], 0.9e5,
                                [np.full(shp, 0.01), np.full(shp, 0.02)])
    r = O.rhs(q, g)
    assert float(r.abs().max()) == 0.0


def test_hydrostatic_rest_is_preserved():
    g, _ = W.bubble_2d()
    rho, p = W.rest_fields(g)
    q = W.state_from_primitives(g, rho, 0.0, 0.0, 0.0, p)
    r = O.rhs(q, g)
    # round-off of p' = p - pbar only (|p| ~ 1e5 Pa)
    assert float(r[0].abs().max()) < 1e-15
    assert float(r[3].abs().max()) < 1e-12
    qn = O.run(q, g, 0.27, 20)
    qi = g.interior(qn.numpy())
    assert np.max(np.abs(qi[1:4] / qi[0])) < 1e-12


def test_conservation_periodic_no_gravity():
    g = W.Grid(nx=16, ny=12, nz=10, dx=100.0, dy=120.0, dz=90.0, grav=0.0, bc=(0, 0, 0), ntracer=1)
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(10, 1.0, 1.0e5)
    q = W.random_smooth_state(g, seed=5)
    s0 = O.conservation_sums(q, g)
    dt = O.cfl_dt(q, g, 0.9)
    qn = O.run(q, g, dt, 10)
    s1 = O.conservation_sums(qn, g)
    scale = np.abs(g.interior(q)).reshape(g.nvar, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale


def test_conservation_with_gravity_and_walls():
    """Mass and x-momentum conserved; total energy changes by exactly the
    Runge-Kutta-weighted gravity work -g sum(rho w) dt (weights 1/6, 1/6, 2/3)."""
    g, q = W.bubble_2d(nx=32, nz=32)
    q = torch.as_tensor(q)
    dt = 0.5
    stages = []

    def f(y):
        stages.append(y.clone())
        return O.rhs(O._with_interior(q, g, y), g)

    qn = O._interior(q, g)
    for _ in range(3):
        stages.clear()
        new = O.rk3(f, qn, dt)
        work = sum(wt * float(-g.grav * s[3].sum()) for wt, s in zip((1 / 6, 1 / 6, 2 / 3), stages))
        dE = float(new[4].sum() - qn[4].sum())
        assert abs(dE - dt * work) <= 1e-12 * float(qn[4].abs().sum())
        assert abs(float(new[0].sum() - qn[0].sum())) <= 1e-14 * float(qn[0].sum())
        assert abs(float(new[1].sum() - qn[1].sum())) <= 1e-14 * float(qn[0].sum()) * 10.0
        qn = new


def test_uniform_tracer_fraction_stays_uniform():
    g, q = W.bubble_2d(nx=32, nz=32)
    g = g.copy(ntracer=2)
    q2 = np.zeros(g.shape)
    q2[:5] = q
    q2[5] = 0.013 * q[0]
    q2[6] = 0.0021 * q[0]
    qn = O.run(q2, g, 0.5, 5).numpy()
    qi = g.interior(qn)
    assert np.max(np.abs(qi[5] / qi[0] - 0.013)) < 1e-15
    assert np.max(np.abs(qi[6] / qi[0] - 0.0021)) < 1e-16


def test_bubble_stays_mirror_symmetric():
    g, q = W.bubble_2d(nx=32, nz=32)
    qn = O.run(q, g, 0.5, 5).numpy()
    qi = g.interior(qn)
    flip = qi[:, :, :, ::-1]
    for m, sgn in ((0, 1), (1, -1), (3, 1), (4, 1)):
        d = np.max(np.abs(qi[m] - sgn * flip[m]))
        assert d <= 1e-12 * max(np.max(np.abs(qi[m])), 1e-30), (m, d)
    assert np.max(np.abs(qi[1])) > 0.0                  # the flow is not trivially zero


def test_cfl_dt_value_and_state_check():
    g, q = W.bubble_2d()
    dt = O.cfl_dt(q, g, 0.9)
    _, p = W.rest_fields(g)
    c = np.sqrt(g.gamma * p / g.interior(q)[0])      # the bubble starts at rest with p = pbar
    assert abs(dt - 0.9 / np.max(c / g.dx + c / g.dz)) <= 1e-9 * dt
    bad = q.copy()
    g.interior(bad)[4, 3, 0, 5] = -1.0
    with pytest.raises(FloatingPointError):
        O.cfl_dt(bad, g, 0.9)
