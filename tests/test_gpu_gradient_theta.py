"""Gradient of a checkpointed multi-segment SSP-RK3 run with respect to the
initial potential-temperature perturbation, against finite differences.

The workload is the gradient benchmark (the convection state with a seeded
smooth flow in the top 16 levels and a smooth pressure perturbation) on a
64 x 64 x 64 grid with the benchmark's spacing (78.125 m), 60 steps of the
initial CFL 0.9 time step, a checkpoint every 20 steps (three segments), and
the loss J = kinetic energy of the top 16 levels. The state is built from
theta' in torch (``workloads.state_from_theta``), so autograd carries the
library's RK3 adjoint (Sec. 4.3, reversed) back to theta'.

Bars:
* the FP64 gradient against Richardson-extrapolated central differences of the
  FP64 forward (steps h = 1e-4 K and h / 2) along 8 seeded directions: relative
  disagreement of <grad J, delta> at most GRAD64_TOL. Where an interface
  velocity crosses zero LMARS switches its upwind side, and differences that
  straddle such a switch carry an error of order h; on this case it measured
  below 4e-6 at h = 1e-4 K (it falls in proportion to h);
* the FP32 gradient (FP32 state and stencil arithmetic, the workload's form)
  within GRAD32_TOL of the FP64 one in the L2 norm over all cells, and its
  directional derivatives within GRAD32_DIR_TOL of the differences;
* the gradient with kept stage states equals the one that recomputes them,
  bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_1901_02955_amd as snap
from paper_1901_02955_amd.autograd import rk3_run
import workloads as wl

pytestmark = pytest.mark.gpu

N, STEPS, EVERY, NDIR = 64, 60, 20, 8
H = 1e-4
GRAD64_TOL = 5e-5
GRAD32_TOL = 1e-2
GRAD32_DIR_TOL = 5e-2
CFL = 0.9


def top_ke(grid, q, levels=16):
    g0 = snap.SNAP_NG
    top = q[:, g0 + grid.nz - levels:g0 + grid.nz, g0:g0 + grid.ny, g0:g0 + grid.nx].double()
    return 0.5 * grid.dx * grid.dy * grid.dz * ((top[1] ** 2 + top[2] ** 2 + top[3] ** 2) / top[0]).sum()


@pytest.fixture(scope="module")
def setup():
    lx = 20e3 * N / 256
    lz = 10e3 * N / 128
    grid, base, dth, vel, dp = wl.convection_flow_3d(N, N, N, lx=lx, ly=lx, lz=lz)
    th0 = torch.as_tensor(dth, device="cuda")
    vd = torch.as_tensor(vel, device="cuda")
    pd = torch.as_tensor(dp, device="cuda")
    dg = {t: snap.device_grid(grid, dtype=t) for t in (torch.float64, torch.float32)}
    with torch.no_grad():
        q = wl.state_from_theta(grid, base, th0, vd, pd)
    dt = snap.snap_cfl_dt(dg[torch.float64], q, CFL,
                          snap.workspace(dg[torch.float64], snap.SNAP_OP_CFL))
    return grid, base, th0, vd, pd, dg, dt


def gradient(setup, dtype, keep=True):
    grid, base, th0, vd, pd, dg, dt = setup
    th = th0.clone().requires_grad_(True)
    q0 = wl.state_from_theta(grid, base, th, vd, pd).to(dtype)
    out = rk3_run(dg[dtype], q0, dt, STEPS, EVERY, keep_stages=keep)
    top_ke(grid, out).backward()
    return th.grad.detach()


def test_gradient_theta_vs_finite_differences(setup):
    grid, base, th0, vd, pd, dg, dt = setup
    print(f"[gradient] {N}^3, {STEPS} steps, checkpoint every {EVERY}, dt {dt:.6g}", flush=True)
    g64 = gradient(setup, torch.float64)
    g32 = gradient(setup, torch.float32)
    g32_re = gradient(setup, torch.float32, keep=False)
    assert torch.equal(g32, g32_re)
    assert torch.isfinite(g64).all() and torch.isfinite(g32).all()
    rel = float((g32.double() - g64).norm() / g64.norm())
    print(f"[gradient] |g32 - g64| / |g64| = {rel:.3e}", flush=True)
    assert rel <= GRAD32_TOL
    work = snap.workspace(dg[torch.float64], snap.SNAP_OP_RK3)

    def loss64(th):
        with torch.no_grad():
            q = wl.state_from_theta(grid, base, th, vd, pd)
            for _ in range(STEPS):
                snap.snap_rk3_step(dg[torch.float64], q, dt, work)
            return float(top_ke(grid, q))

    e64, e32 = [], []
    for s in range(5, 5 + NDIR):
        d = torch.as_tensor(wl.seeded_normal((N, N, N), s), device="cuda")

        def central(h):
            return (loss64(th0 + h * d) - loss64(th0 - h * d)) / (2.0 * h)

        fd = (4.0 * central(0.5 * H) - central(H)) / 3.0
        a64 = float((g64 * d).sum())
        a32 = float((g32.double() * d).sum())
        e64.append(abs(a64 - fd) / max(abs(a64), abs(fd)))
        e32.append(abs(a32 - fd) / max(abs(a32), abs(fd)))
        print(f"[gradient] seed {s}: FD {fd:.10e} AD64 {a64:.10e} ({e64[-1]:.2e}) "
              f"AD32 {a32:.10e} ({e32[-1]:.2e})", flush=True)
    assert max(e64) <= GRAD64_TOL, e64
    assert max(e32) <= GRAD32_DIR_TOL, e32
