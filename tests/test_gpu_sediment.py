"""GPU parity of the sedimentation of condensates (Sec. 2, eq. d3 and the
momentum and total-energy equations with terminal velocities) against the
FP64 CPU oracle: right-hand side within 1e-12 per field (FP64) and 1e-4
(FP32 form), three RK3 steps within the multi-step bar, with walls (no
inflow through the lid, outflow through the ground) and periodic in z.

The adjoint with falling condensates (k_adj_sediment after the direction
kernels) against the oracle's autograd: right-hand side within 1e-11 (FP64)
and 1e-4 (FP32 at the same FP32-rounded inputs), one RK3 step within 1e-11;
the sedimentation's share of the oracle's J^T r_bar is 1e-3 to 2e-2 of the
density and condensate fields (1e-7 of the momenta), far above those bars."""
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


@pytest.fixture(scope="module")
def scases():
    return {n: C.build_sediment_case(n, s) for n, s in C.SED_SPECS}


@pytest.mark.parametrize("name", C.SED_NAMES)
def test_rhs_fp64_sediment(scases, name):
    c = scases[name]
    print(f"[sediment] rhs fp64 {name}", flush=True)
    dg = snap.device_grid(c.grid)
    qd = torch.as_tensor(c.q).cuda()
    rhs = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    ref = oracle.rhs(c.q, c.grid).numpy()
    errs = field_errors(rhs.cpu().numpy(), ref)
    # the sedimentation part is not negligible: compare with the rain at rest
    ref0 = oracle.rhs(c.q, c.grid.copy(tracer_wt=(0.0,) * c.grid.ntracer)).numpy()
    share = float(np.max(np.abs(ref[9] - ref0[9])) / np.max(np.abs(ref[9])))
    print("   errors", ["%.2e" % e for e in errs], "rain share %.2f" % share, flush=True)
    assert all(e <= TOL64 for e in errs), errs
    assert share > 0.05


@pytest.mark.parametrize("name", C.SED_NAMES)
def test_rk3_steps_fp64_sediment(scases, name):
    c = scases[name]
    print(f"[sediment] rk3 fp64 {name}", flush=True)
    dg = snap.device_grid(c.grid)
    qd = torch.as_tensor(c.q).cuda()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    for _ in range(3):
        snap.snap_rk3_step(dg, qd, c.dt, work)
    ref, kappa = rounding_sensitivity(c.grid, c.q, c.dt, 3)
    assert_steps_close(c.grid.interior(qd.cpu().numpy()), ref, kappa, f"{name}, 3 steps")


@pytest.mark.parametrize("name", C.SED_NAMES)
def test_rhs_fp32_sediment(scases, name):
    c = scases[name]
    q32 = torch.as_tensor(c.q).float()
    dg = snap.device_grid(c.grid, dtype=torch.float32)
    rhs = torch.empty(dg.interior_shape, dtype=torch.float32, device="cuda")
    snap.snap_rhs(dg, q32.cuda(), rhs)
    ref = oracle.rhs(q32.double().numpy(), c.grid).numpy()
    errs = field_errors(rhs.cpu().double().numpy(), ref)
    print(f"[sediment] fp32 {name}", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= RHS32_TOL for e in errs), errs


@pytest.mark.parametrize("name", C.SED_NAMES)
def test_rhs_adjoint_sediment(scases, name):
    c = scases[name]
    print(f"[sediment] adjoint {name}", flush=True)
    rbar = wl.seeded_normal(c.grid.interior_shape, 150)
    ref = oracle.rhs_adjoint(c.q, c.grid, rbar).numpy()
    dg = snap.device_grid(c.grid)
    qb = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    snap.snap_rhs_adjoint(dg, torch.as_tensor(c.q).cuda(), torch.as_tensor(rbar).cuda(), qb,
                          snap.workspace(dg, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qb.cpu().numpy(), ref)
    print("   FP64", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
    q32 = c.q.astype(np.float32).astype(np.float64)
    r32 = rbar.astype(np.float32).astype(np.float64)
    ref32 = oracle.rhs_adjoint(q32, c.grid, r32).numpy()
    dg32 = snap.device_grid(c.grid, dtype=torch.float32)
    qbf = torch.empty(dg32.interior_shape, dtype=torch.float32, device="cuda")
    snap.snap_rhs_adjoint(dg32, torch.as_tensor(q32).float().cuda(), torch.as_tensor(r32).float().cuda(),
                          qbf, snap.workspace(dg32, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qbf.cpu().double().numpy(), ref32)
    print("   FP32", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-4 for e in errs), errs


@pytest.mark.parametrize("name", C.SED_NAMES)
def test_rk3_step_adjoint_sediment(scases, name):
    c = scases[name]
    print(f"[sediment] rk3 adjoint {name}", flush=True)
    qbar = wl.seeded_normal(c.grid.interior_shape, 151)
    ref = oracle.rk3_step_adjoint(c.q, c.grid, c.dt, qbar).numpy()
    dg = snap.device_grid(c.grid)
    qb = torch.as_tensor(qbar).cuda()
    snap.snap_rk3_step_adjoint(dg, torch.as_tensor(c.q).cuda(), c.dt, qb,
                               snap.workspace(dg, snap.SNAP_OP_RK3_ADJ))
    errs = field_errors(qb.cpu().numpy(), ref)
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
