"""Order of accuracy of the whole oracle right-hand side and step on an
advected density wave (uniform velocity and pressure, no gravity): the
right-hand side converges at fifth order (WENO5, Sec. 4.2) and full steps
with dt ~ h^(5/3) at fifth order overall (TVD-RK3, Sec. 4.3)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O

AMP = 0.2


def _wave_grid(n, axis):
    dims = [1, 1, 1]
    dims[axis] = n
    nx, ny, nz = dims
    h = 1.0 / n
    g = W.Grid(nx=nx, ny=ny, nz=nz, dx=h if axis == 0 else 1.0, dy=h if axis == 1 else 1.0,
               dz=h if axis == 2 else 1.0, gamma=1.4, grav=0.0, bc=(0, 0, 0))
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(nz, 1.0, 1.0)
    return g, h


def _wave_state(n, axis, shift=0.0):
    g, h = _wave_grid(n, axis)
    edges = np.arange(n + 1) * h - shift
    avg = 1.0 + AMP * (np.cos(2 * np.pi * edges[:-1]) - np.cos(2 * np.pi * edges[1:])) / (2 * np.pi * h)
    shp = [1, 1, 1]
    shp[2 - axis] = n
    rho = avg.reshape(shp)
    vel = [0.0, 0.0, 0.0]
    vel[axis] = 1.0
    q = W.state_from_primitives(g, rho, vel[0], vel[1], vel[2], 1.0)
    return g, h, q


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rhs_fifth_order_on_density_wave(axis):
    errs = []
    ns = (32, 64, 128, 256)
    for n in ns:
        g, h, q = _wave_state(n, axis)
        r = O.rhs(q, g)[0].reshape(-1).numpy()
        x = np.arange(n + 1) * h
        exact = -1.0 * AMP * (np.sin(2 * np.pi * x[1:]) - np.sin(2 * np.pi * x[:-1])) / h
        errs.append(np.max(np.abs(r - exact)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert min(orders) >= 4.7, orders


def test_full_steps_fifth_order_with_dt_h_five_thirds():
    tend = 0.1
    errs = []
    ns = (32, 64, 128)
    for n in ns:
        g, h, q = _wave_state(n, 0)
        nsteps = int(math.ceil(tend / h ** (5.0 / 3.0)))
        dt = tend / nsteps
        qn = torch.as_tensor(q)
        for _ in range(nsteps):
            qn = O.rk3_step(qn, g, dt)
        _, _, qex = _wave_state(n, 0, shift=tend)
        errs.append(np.max(np.abs(g.interior(qn.numpy())[0] - g.interior(qex)[0])))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert min(orders) >= 4.7, orders
