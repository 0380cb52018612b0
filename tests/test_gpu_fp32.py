"""GPU parity of the FP32 form against the FP64 CPU oracle.

The FP32 form stores the state and runs the stencil arithmetic in single
precision, keeping double precision for the hydrostatic reference and the
E -> p inversion. Bars:
* after 100 SSP-RK3 steps of a seeded 3-D convection case, density and total
  energy within 1e-5 of the oracle, relative to the largest magnitude of the
  field (the FP32 tolerance of the method's specification); the per-field max
  and L2 errors of every field are printed;
* a single right-hand side within RHS32_TOL per field, relative to the largest
  magnitude of the field: FP32 rounding of fluxes of size F over a cell of
  size dx leaves about 1e-7 F / dx, a few 1e-6 of the divergence on these
  cases; the bar keeps a factor of 10 over the largest error seen.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
import workloads as wl
from tests import cases as C
from tests.test_gpu_parity import field_errors

pytestmark = pytest.mark.gpu

RHS32_TOL = 1e-4
STATE32_TOL = 1e-5


@pytest.mark.parametrize("name", C.CASE_NAMES)
def test_rhs_fp32(name):
    c = C.build_case(name, dict(C.SPECS)[name])
    print(f"[fp32] rhs {name}", flush=True)
    dg = snap.device_grid(c.grid, dtype=torch.float32)
    q32 = torch.as_tensor(c.q).float()
    qd = q32.cuda()
    rhs = torch.empty(dg.interior_shape, dtype=torch.float32, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    # the oracle sees the same (FP32-rounded) input state
    ref = oracle.rhs(q32.double().numpy(), c.grid).numpy()
    errs = field_errors(rhs.cpu().double().numpy(), ref)
    print("   per-field max error / max|field|:", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= RHS32_TOL for e in errs), errs


def test_fp32_100_steps_convection():
    grid, q, _ = wl.convection_3d(24, 20, 32, lx=20e3 * 24 / 256, ly=20e3 * 20 / 256,
                                  lz=10e3 * 32 / 128, seed=9)
    # stronger noise so the flow develops within 100 steps
    rng = np.random.default_rng(10)
    qi = grid.interior(q)
    qi[1:4] = qi[0] * rng.uniform(-2.0, 2.0, size=qi[1:4].shape)
    qi[4] = qi[4] + 0.5 * (qi[1] ** 2 + qi[2] ** 2 + qi[3] ** 2) / qi[0]
    # both sides start from the FP32-rounded state, so that the comparison
    # measures the FP32 form's arithmetic and storage, not input rounding
    q = q.astype(np.float32).astype(np.float64)
    dt = 0.5 * oracle.cfl_dt(q, grid, 0.9)
    nsteps = 100
    print("[fp32] 100 steps 24x20x32", flush=True)
    ref = grid.interior(oracle.run(q, grid, dt, nsteps).numpy())
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = torch.as_tensor(q).float().cuda()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    for _ in range(nsteps):
        snap.snap_rk3_step(dg, qd, dt, work)
    got = grid.interior(qd.cpu().double().numpy())
    names = ["rho", "rho u", "rho v", "rho w", "E"]
    # deviation of the oracle's state from the hydrostatic base (what the flow
    # has developed): the second normalisation of the per-field errors
    base = np.zeros_like(ref)
    base[0] = grid.rhobar_cell[3:3 + grid.nz][:, None, None]
    base[4] = grid.pbar_cell[3:3 + grid.nz][:, None, None] / (grid.gamma - 1.0)
    for v in range(grid.nvar):
        d = got[v] - ref[v]
        dev = ref[v] - base[v]
        print(f"   {names[v]:6s} max {np.abs(d).max() / np.abs(ref[v]).max():.3e}  "
              f"L2 {np.sqrt((d ** 2).mean()) / np.sqrt((ref[v] ** 2).mean()):.3e}  "
              f"max/dev {np.abs(d).max() / np.abs(dev).max():.3e}", flush=True)
    errs = field_errors(got, ref)
    assert errs[0] <= STATE32_TOL and errs[4] <= STATE32_TOL, errs
