"""GPU parity of the mixture equation of state (Sec. 2, eq. eos; App. B, eq. p2
and the effective adiabatic index) against the FP64 CPU oracle.

Same bars as the passive path: right-hand side within 1e-12 per field
(relative to the field's largest magnitude), states after several steps
within max(1e-12, 10 x the oracle's own 1-ulp input sensitivity), CFL step
within 4 ulp, FP32 right-hand side within 1e-4. Also: the mixture reduces
to the passive path when every vapour's heat-capacity ratio is 1/eps and there
is no condensate or chemical energy; the right-hand-side and RK3 adjoints
match the oracle's autograd (FP64 1e-11, FP32 1e-4).
"""
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
def mix_cases():
    return {n: C.build_case(n, s) for n, s in C.MIX_SPECS}


def gpu_state(grid, q, dtype=torch.float64):
    dg = snap.device_grid(grid, dtype=dtype)
    assert dg.eos == snap.SNAP_EOS_MIXTURE
    return dg, torch.as_tensor(q).to(dtype).cuda().contiguous()


@pytest.mark.parametrize("name", C.MIX_NAMES)
def test_rhs_fp64_mixture(mix_cases, name):
    c = mix_cases[name]
    print(f"[moist] rhs fp64 {name}", flush=True)
    dg, qd = gpu_state(c.grid, c.q)
    rhs = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    errs = field_errors(rhs.cpu().numpy(), oracle.rhs(c.q, c.grid).numpy())
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= TOL64 for e in errs), errs


@pytest.mark.parametrize("name", C.MIX_NAMES)
def test_rk3_steps_fp64_mixture(mix_cases, name):
    c = mix_cases[name]
    print(f"[moist] rk3 fp64 {name}", flush=True)
    dg, qd = gpu_state(c.grid, c.q)
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    nsteps = 3
    for _ in range(nsteps):
        snap.snap_rk3_step(dg, qd, c.dt, work)
    ref, kappa = rounding_sensitivity(c.grid, c.q, c.dt, nsteps)
    got = c.grid.interior(qd.cpu().numpy())
    assert_steps_close(got, ref, kappa, f"{name}, {nsteps} steps")


@pytest.mark.parametrize("name", C.MIX_NAMES)
def test_cfl_dt_mixture(mix_cases, name):
    c = mix_cases[name]
    dg, qd = gpu_state(c.grid, c.q)
    dt = snap.snap_cfl_dt(dg, qd, 0.9, snap.workspace(dg, snap.SNAP_OP_CFL))
    ref = oracle.cfl_dt(c.q, c.grid, 0.9)
    print(f"[moist] cfl {name}: {dt!r} vs {ref!r}", flush=True)
    assert abs(dt - ref) <= 4 * np.spacing(ref)


@pytest.mark.parametrize("name", C.MIX_NAMES)
def test_rhs_fp32_mixture(mix_cases, name):
    c = mix_cases[name]
    print(f"[moist] rhs fp32 {name}", flush=True)
    q32 = torch.as_tensor(c.q).float()
    dg, qd = gpu_state(c.grid, c.q, torch.float32)
    rhs = torch.empty(dg.interior_shape, dtype=torch.float32, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    ref = oracle.rhs(q32.double().numpy(), c.grid).numpy()
    errs = field_errors(rhs.cpu().double().numpy(), ref)
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= RHS32_TOL for e in errs), errs


def test_mixture_reduces_to_passive_on_gpu():
    """Vapours with sigma = 1/eps, no condensates, no chemical energy: the two
    equations of state give the same right-hand side (the kernels differ only
    in rounding order)."""
    c = C.build_case("3d_tracers_20x18x24_nt4", dict(C.SPECS)["3d_tracers_20x18x24_nt4"])
    species = [(wl.TRACER_VAPOUR, e, 1.0 / e, 0.0) for e in (7.8, 7.4, 3.1, 0.5)]
    gm = wl.with_mixture(c.grid, species)
    dp = snap.device_grid(c.grid)
    dm = snap.device_grid(gm)
    qd = torch.as_tensor(c.q).cuda()
    rp = torch.empty(dp.interior_shape, dtype=torch.float64, device="cuda")
    rm = torch.empty_like(rp)
    snap.snap_rhs(dp, qd, rp)
    snap.snap_rhs(dm, qd, rm)
    errs = field_errors(rm.cpu().numpy(), rp.cpu().numpy())
    print("[moist] passive reduction", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-13 for e in errs), errs


def test_mixture_rhs_deterministic(mix_cases):
    c = mix_cases["mix_3d_25x19x22_nt4"]
    dg, qd = gpu_state(c.grid, c.q)
    r1 = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    r2 = torch.empty_like(r1)
    snap.snap_rhs(dg, qd, r1)
    snap.snap_rhs(dg, qd, r2)
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("name", C.MIX_NAMES)
def test_rhs_adjoint_mixture(mix_cases, name):
    """The right-hand-side adjoint under the mixture equation of state (the
    reverse of the mixture LMARS flux and of the mixture conserved -> primitive
    map) against the oracle's autograd: FP64 within 1e-11, FP32 within 1e-4 at
    the same FP32-rounded inputs."""
    c = mix_cases[name]
    print(f"[moist] adjoint {name}", flush=True)
    rbar = wl.seeded_normal(c.grid.interior_shape, 140)
    ref = oracle.rhs_adjoint(c.q, c.grid, rbar).numpy()
    dg, qd = gpu_state(c.grid, c.q)
    rb = torch.as_tensor(rbar).cuda()
    qb = torch.empty_like(rb)
    snap.snap_rhs_adjoint(dg, qd, rb, qb, snap.workspace(dg, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qb.cpu().numpy(), ref)
    print("   FP64", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
    q32 = c.q.astype(np.float32).astype(np.float64)
    r32 = rbar.astype(np.float32).astype(np.float64)
    ref32 = oracle.rhs_adjoint(q32, c.grid, r32).numpy()
    dg32, q32d = gpu_state(c.grid, q32, torch.float32)
    rbf = torch.as_tensor(r32).float().cuda()
    qbf = torch.empty_like(rbf)
    snap.snap_rhs_adjoint(dg32, q32d, rbf, qbf, snap.workspace(dg32, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qbf.cpu().double().numpy(), ref32)
    print("   FP32", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-4 for e in errs), errs


def test_rk3_step_adjoint_mixture(mix_cases):
    c = mix_cases[C.MIX_NAMES[0]]
    qbar = wl.seeded_normal(c.grid.interior_shape, 141)
    ref = oracle.rk3_step_adjoint(c.q, c.grid, c.dt, qbar).numpy()
    dg, qd = gpu_state(c.grid, c.q)
    qb = torch.as_tensor(qbar).cuda()
    snap.snap_rk3_step_adjoint(dg, qd, c.dt, qb, snap.workspace(dg, snap.SNAP_OP_RK3_ADJ))
    errs = field_errors(qb.cpu().numpy(), ref)
    print("[moist] rk3 adjoint", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs
