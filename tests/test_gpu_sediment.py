"""GPU parity of the sedimentation of condensates (Sec. 2, eq. d3 and the
momentum and total-energy equations with terminal velocities) against the
FP64 CPU oracle: right-hand side within 1e-12 per field (FP64) and 1e-4
(FP32 form), three RK3 steps within the multi-step bar, with walls (no
inflow through the lid, outflow through the ground) and periodic in z."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
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
