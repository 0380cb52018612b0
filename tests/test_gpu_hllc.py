"""GPU parity of the HLLC Riemann solver (the paper's alternative to LMARS)
against the FP64 CPU oracle, on the passive parity cases: right-hand side
within 1e-12 per field (FP64) and 1e-4 (FP32 form), three RK3 steps within
the multi-step bar, and determinism.

In the star region HLLC's fluxes are F + S (U* - U), differences of terms of
size S U; for the state at rest (the bubble) the mass and energy right-hand
sides are pure rounding of those terms, so for that case alone the FP64 bar
carries an absolute floor at that rounding: 1e-15 c_max max|U_m| /
min(dx, dy, dz). Every case in motion is held to the relative bar alone."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
import workloads as wl
from tests import cases as C
from tests.test_gpu_fp32 import RHS32_TOL
from tests.test_gpu_parity import TOL64, assert_steps_close, field_errors, rounding_sensitivity

pytestmark = pytest.mark.gpu

HLLC_CASES = ["2d_bubble_64x64", "2d_smooth_37x29_nt3", "2d_reflect_21x19", "2d_thin_19x2",
              "3d_smooth_35x21x19", "3d_tracers_20x18x24_nt4", "3d_linear_17x9x11",
              "3d_periodic_z_12x10x14", "3d_small_2x3x4", "3d_xwall_19x17x12",
              "3d_periodic_all_13x11x10"]


@pytest.fixture(scope="module")
def hcases():
    out = {}
    for n in HLLC_CASES:
        c = C.build_case(n, dict(C.SPECS)[n])
        out[n] = C.Case(n, c.grid.copy(riemann=wl.RIEMANN_HLLC), c.q, c.dt)
    return out


@pytest.mark.parametrize("name", HLLC_CASES)
def test_rhs_fp64_hllc(hcases, name):
    c = hcases[name]
    print(f"[hllc] rhs fp64 {name}", flush=True)
    dg = snap.device_grid(c.grid)
    rhs = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    snap.snap_rhs(dg, torch.as_tensor(c.q).cuda(), rhs)
    got, ref = rhs.cpu().numpy(), oracle.rhs(c.q, c.grid).numpy()
    qi = c.grid.interior(c.q)
    cmax = float(np.max(np.sqrt(c.grid.gamma * 0.4 * qi[4] / qi[0]))) * 2.0   # generous c bound
    dmin = min(c.grid.dx, c.grid.dz, c.grid.dy if c.grid.ny > 1 else c.grid.dx)
    # the rounding floor is for the state at rest only (the bubble, whose mass
    # and energy right-hand sides are pure rounding of the star-region terms);
    # every case in motion is held to the relative bar alone
    at_rest = name == "2d_bubble_64x64"
    bad = []
    for m in range(c.grid.nvar):
        floor = 1e-15 * cmax * float(np.max(np.abs(qi[m]))) / dmin if at_rest else 0.0
        err = float(np.max(np.abs(got[m] - ref[m])))
        bar = TOL64 * float(np.max(np.abs(ref[m]))) + floor
        print(f"   field {m}: error {err:.2e}  bar {bar:.2e}", flush=True)
        if not err <= bar:
            bad.append(m)
    assert not bad, bad


@pytest.mark.parametrize("name", ["2d_bubble_64x64", "3d_smooth_35x21x19", "3d_tracers_20x18x24_nt4"])
def test_rk3_fp64_hllc(hcases, name):
    c = hcases[name]
    print(f"[hllc] rk3 fp64 {name}", flush=True)
    dg = snap.device_grid(c.grid)
    qd = torch.as_tensor(c.q).cuda()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    for _ in range(3):
        snap.snap_rk3_step(dg, qd, c.dt, work)
    ref, kappa = rounding_sensitivity(c.grid, c.q, c.dt, 3)
    assert_steps_close(c.grid.interior(qd.cpu().numpy()), ref, kappa, f"hllc {name}")


@pytest.mark.parametrize("name", ["2d_smooth_37x29_nt3", "3d_smooth_35x21x19", "3d_tracers_20x18x24_nt4"])
def test_rhs_fp32_hllc(hcases, name):
    c = hcases[name]
    q32 = torch.as_tensor(c.q).float()
    dg = snap.device_grid(c.grid, dtype=torch.float32)
    rhs = torch.empty(dg.interior_shape, dtype=torch.float32, device="cuda")
    snap.snap_rhs(dg, q32.cuda(), rhs)
    errs = field_errors(rhs.cpu().double().numpy(), oracle.rhs(q32.double().numpy(), c.grid).numpy())
    print(f"[hllc] fp32 {name}", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= RHS32_TOL for e in errs), errs


def test_hllc_differs_from_lmars_and_is_deterministic(hcases):
    c = hcases["3d_smooth_35x21x19"]
    qd = torch.as_tensor(c.q).cuda()
    dh = snap.device_grid(c.grid)
    dl = snap.device_grid(c.grid.copy(riemann=wl.RIEMANN_LMARS))
    rh = torch.empty(dh.interior_shape, dtype=torch.float64, device="cuda")
    rh2, rl = torch.empty_like(rh), torch.empty_like(rh)
    snap.snap_rhs(dh, qd, rh)
    snap.snap_rhs(dh, qd, rh2)
    snap.snap_rhs(dl, qd, rl)
    assert torch.equal(rh, rh2)
    assert float((rh[0] - rl[0]).abs().max()) > 1e-3 * float(rl[0].abs().max())


# The adjoint with the HLLC flux (the reverse of hllc_flux in the direction
# kernels): against the oracle's autograd through its HLLC right-hand side, on
# the cases in motion (at rest the star region's branch and the outer-speed
# selections follow rounding, as LMARS's upwind side does in the FP64 adjoint
# tests).
ADJ_HLLC = ["2d_smooth_37x29_nt3", "2d_reflect_21x19", "3d_smooth_35x21x19",
            "3d_tracers_20x18x24_nt4", "3d_linear_17x9x11", "3d_periodic_z_12x10x14",
            "3d_small_2x3x4", "3d_xwall_19x17x12"]


@pytest.mark.parametrize("name", ADJ_HLLC)
def test_rhs_adjoint_hllc(hcases, name):
    c = hcases[name]
    print(f"[hllc] adjoint {name}", flush=True)
    rbar = wl.seeded_normal(c.grid.interior_shape, 130)
    ref = oracle.rhs_adjoint(c.q, c.grid, rbar).numpy()
    dg = snap.device_grid(c.grid)
    qd = torch.as_tensor(c.q).cuda()
    rb = torch.as_tensor(rbar).cuda()
    qb = torch.empty_like(rb)
    work = snap.workspace(dg, snap.SNAP_OP_RHS_ADJ)
    snap.snap_rhs_adjoint(dg, qd, rb, qb, work)
    errs = field_errors(qb.cpu().numpy(), ref)
    print("   FP64", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
    # single precision (the march for y and z) at the same FP32-rounded inputs
    q32 = c.q.astype(np.float32).astype(np.float64)
    r32 = rbar.astype(np.float32).astype(np.float64)
    ref32 = oracle.rhs_adjoint(q32, c.grid, r32).numpy()
    dg32 = snap.device_grid(c.grid, dtype=torch.float32)
    rbf = torch.as_tensor(r32).float().cuda()
    qbf = torch.empty_like(rbf)
    snap.snap_rhs_adjoint(dg32, torch.as_tensor(q32).float().cuda(), rbf, qbf,
                          snap.workspace(dg32, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qbf.cpu().double().numpy(), ref32)
    print("   FP32", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-4 for e in errs), errs


@pytest.mark.parametrize("name", ["2d_smooth_37x29_nt3", "3d_smooth_35x21x19"])
def test_rk3_step_adjoint_hllc(hcases, name):
    c = hcases[name]
    qbar = wl.seeded_normal(c.grid.interior_shape, 131)
    ref = oracle.rk3_step_adjoint(c.q, c.grid, c.dt, qbar).numpy()
    dg = snap.device_grid(c.grid)
    qd = torch.as_tensor(c.q).cuda()
    qb = torch.as_tensor(qbar).cuda()
    snap.snap_rk3_step_adjoint(dg, qd, c.dt, qb, snap.workspace(dg, snap.SNAP_OP_RK3_ADJ))
    errs = field_errors(qb.cpu().numpy(), ref)
    print(f"[hllc] rk3 adjoint {name}", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
