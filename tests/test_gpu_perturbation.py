"""Perturbation storage (SNAP_STORE_PERTURBATION): q holds rho - rhobar_k and
E - pbar_k / (gamma - 1) in place of rho and E.

Every entry point must compute what it computes for the full state: the
oracle works on the full state, and the tests convert with
``workloads.to_perturbation`` / ``from_perturbation`` on the host in FP64.
Bars (FP64):
* right-hand side within 1e-12 per field of the oracle's, relative to the
  field's largest magnitude (the bar of the full state; the stored density
  and energy are rounded once more, rho = rho' + rhobar, a few ulp);
* one RK3 step, back in full form, within 1e-11 per field (the smooth cases,
  where every term is active and no flow grows out of round-off);
* the CFL time step within 1e-14 relative and the conservation sums within
  1e-13 of the oracle's (relative to the sum of magnitudes);
* the right-hand-side adjoint within 1e-11 of the oracle's (the Jacobian does
  not depend on the storage form);
* the device-dt steps and the batched step agree with the full-state path.
FP32: after 100 steps of a convection case both storage forms keep rho and E
within 1e-5 of the oracle, and the perturbation form keeps every field at
least as close as the full form (the full form rounds E of about 1e5 J/m^3 to
single precision at every stage).
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

PERT = snap.SNAP_STORE_PERTURBATION
NAMES = ["2d_smooth_37x29_nt3", "2d_reflect_21x19", "3d_smooth_35x21x19", "3d_tracers_20x18x24_nt4",
         "3d_xwall_19x17x12", "3d_periodic_all_13x11x10", "3d_small_2x3x4"]


def case(name):
    return C.build_case(name, dict(C.SPECS)[name])


@pytest.mark.parametrize("name", NAMES)
def test_rhs_fp64(name):
    c = case(name)
    print(f"[pert] rhs {name}", flush=True)
    dg = snap.device_grid(c.grid, storage=PERT)
    qd = torch.as_tensor(wl.to_perturbation(c.grid, c.q)).cuda()
    rhs = torch.empty(dg.interior_shape, dtype=torch.float64, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    errs = field_errors(rhs.cpu().numpy(), oracle.rhs(c.q, c.grid).numpy())
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-12 for e in errs), errs


@pytest.mark.parametrize("name", NAMES)
def test_rk3_step_cfl_sums_fp64(name):
    c = case(name)
    g = c.grid
    print(f"[pert] rk3 {name}", flush=True)
    dg = snap.device_grid(g, storage=PERT)
    qd = torch.as_tensor(wl.to_perturbation(g, c.q)).cuda()
    dt = snap.snap_cfl_dt(dg, qd, 0.9, snap.workspace(dg, snap.SNAP_OP_CFL))
    dt_ref = oracle.cfl_dt(c.q, g, 0.9)
    assert abs(dt - dt_ref) <= 1e-14 * dt_ref, (dt, dt_ref)
    sums = snap.snap_conservation_sums(dg, qd, snap.workspace(dg, snap.SNAP_OP_SUMS))
    vals = g.interior(c.q).reshape(g.nvar, -1)
    assert np.all(np.abs(sums - vals.sum(axis=1)) <= 1e-13 * np.abs(vals).sum(axis=1))
    snap.snap_rk3_step(dg, qd, dt_ref, snap.workspace(dg, snap.SNAP_OP_RK3))
    got = g.interior(wl.from_perturbation(g, qd.cpu().numpy()))
    ref = g.interior(oracle.rk3_step(c.q, g, dt_ref).numpy())
    errs = field_errors(got, ref)
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs


@pytest.mark.parametrize("name", ["2d_smooth_37x29_nt3", "3d_smooth_35x21x19", "3d_tracers_20x18x24_nt4"])
def test_rhs_adjoint_fp64(name):
    c = case(name)
    print(f"[pert] adjoint {name}", flush=True)
    rbar = wl.seeded_normal(c.grid.interior_shape, 110)
    dg = snap.device_grid(c.grid, storage=PERT)
    qd = torch.as_tensor(wl.to_perturbation(c.grid, c.q)).cuda()
    rb = torch.as_tensor(rbar).cuda()
    qb = torch.empty_like(rb)
    snap.snap_rhs_adjoint(dg, qd, rb, qb, snap.workspace(dg, snap.SNAP_OP_RHS_ADJ))
    errs = field_errors(qb.cpu().numpy(), oracle.rhs_adjoint(c.q, c.grid, rbar).numpy())
    print("   errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-11 for e in errs), errs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_device_dt_steps_match_full_state(dtype):
    """snap_rk3_steps_cfl on the stored perturbation against the full state:
    the same time steps (to rounding of rho and p) and the same states."""
    g, _ = wl.dry_grid(37, 23, 19, 7400.0, 4600.0, 2850.0)
    q = wl.random_smooth_state(g, 43)
    n = 4
    out = {}
    for st in (snap.SNAP_STORE_TOTAL, PERT):
        dg = snap.device_grid(g, dtype=dtype, storage=st)
        qq = wl.to_perturbation(g, q) if st == PERT else q
        qd = torch.as_tensor(qq).to(dtype).cuda()
        w = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
        dts = torch.zeros(n, dtype=torch.float64, device="cuda")
        snap.snap_rk3_steps_cfl(dg, qd, 0.9, n, w, dts)
        snap.snap_rk3_steps_status(dg, w)
        full = qd.double().cpu().numpy()
        if st == PERT:
            full = wl.from_perturbation(g, full)
        out[st] = (dts.cpu().numpy(), g.interior(full))
    (d0, s0), (d1, s1) = out[snap.SNAP_STORE_TOTAL], out[PERT]
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert np.all(np.abs(d0 - d1) <= tol * d0), (d0, d1)
    errs = field_errors(s1, s0)
    print(f"[pert] device dt {dtype}: dt {d0[0]:.6g}, state errors", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= (1e-11 if dtype == torch.float64 else 1e-4) for e in errs), errs


def test_batched_step_matches_full_state():
    """Six 2-D members of two sizes in smooth states with every term active
    (bubbles at rest would leave rho u at round-off size after one step)."""
    members = []
    for m, (nx, nz) in enumerate(((64, 48), (40, 24), (64, 48), (40, 24), (40, 24), (64, 48))):
        gm, _ = wl.dry_grid(nx, 1, nz, 200.0 * nx, 200.0, 150.0 * nz, bc=(0, 0, 1))
        members.append((gm, wl.random_smooth_state(gm, 60 + m)))
    grids_t = [snap.device_grid(gm) for gm, _ in members]
    grids_p = [snap.device_grid(gm, storage=PERT) for gm, _ in members]
    qt = [torch.as_tensor(q).cuda() for _, q in members]
    qp = [torch.as_tensor(wl.to_perturbation(gm, q)).cuda() for gm, q in members]
    dts = [0.5 * oracle.cfl_dt(q, gm, 0.9) for gm, q in members]
    snap.snap_rk3_step_batched(grids_t, qt, dts, snap.batched_workspace(grids_t))
    snap.snap_rk3_step_batched(grids_p, qp, dts, snap.batched_workspace(grids_p))
    for (gm, _), a, b in zip(members, qt, qp):
        full = gm.interior(wl.from_perturbation(gm, b.cpu().numpy()))
        errs = field_errors(full, gm.interior(a.cpu().numpy()))
        print("[pert] batched member errors", ["%.2e" % e for e in errs], flush=True)
        assert all(e <= 1e-12 for e in errs), errs


def test_fp32_100_steps_perturbation_storage_is_closer():
    grid, q, _ = wl.convection_3d(24, 20, 32, lx=20e3 * 24 / 256, ly=20e3 * 20 / 256,
                                  lz=10e3 * 32 / 128, seed=9)
    rng = np.random.default_rng(10)
    qi = grid.interior(q)
    qi[1:4] = qi[0] * rng.uniform(-2.0, 2.0, size=qi[1:4].shape)
    qi[4] = qi[4] + 0.5 * (qi[1] ** 2 + qi[2] ** 2 + qi[3] ** 2) / qi[0]
    nsteps = 100
    errs = {}
    for st in (snap.SNAP_STORE_TOTAL, PERT):
        # each form starts from its own FP32 rounding, and the oracle from the
        # same state, so input rounding does not enter
        stored = wl.to_perturbation(grid, q) if st == PERT else q
        s32 = stored.astype(np.float32).astype(np.float64)
        start = wl.from_perturbation(grid, s32) if st == PERT else s32
        dt = 0.5 * oracle.cfl_dt(start, grid, 0.9)
        ref = grid.interior(oracle.run(start, grid, dt, nsteps).numpy())
        dg = snap.device_grid(grid, dtype=torch.float32, storage=st)
        qd = torch.as_tensor(s32).float().cuda()
        work = snap.workspace(dg, snap.SNAP_OP_RK3)
        for _ in range(nsteps):
            snap.snap_rk3_step(dg, qd, dt, work)
        got = qd.cpu().double().numpy()
        if st == PERT:
            got = wl.from_perturbation(grid, got)
        errs[st] = field_errors(grid.interior(got), ref)
        print(f"[pert] fp32 100 steps, storage {st}:", ["%.2e" % e for e in errs[st]], flush=True)
        assert errs[st][0] <= 1e-5 and errs[st][4] <= 1e-5, errs[st]
    assert all(p <= t for p, t in zip(errs[PERT], errs[snap.SNAP_STORE_TOTAL])), errs
