"""snap_rk3_step_cfl against snap_cfl_dt followed by snap_rk3_step.

The device-side step forms dt = cfl / (maximum signal speed) in each stage
kernel with the same double division the host makes, so the two paths must
agree bit for bit, and the dt it reports must equal the host's. Cases: a
ragged 3-D dry grid (double), a 2-D bubble (both element types), the Jovian
column under the mixture equation of state (single), the same with falling
precipitation (the sedimentation kernel reads the device dt too), and the
full 256 x 256 x 128 convection grid (the launch whose chunks are sized per
dispatch pass), three steps each. The state flag that the device-dt calls
leave for snap_rk3_steps_status is tested on a planted negative energy.
"""
import numpy as np
import pytest
import torch

import paper_1901_02955_amd as snap
import workloads as wl

pytestmark = pytest.mark.gpu

CFL = 0.9


def cases():
    g3, _ = wl.dry_grid(37, 23, 19, 7400.0, 4600.0, 2850.0)
    yield "dry_3d_37x23x19_f64", g3, wl.random_smooth_state(g3, 31), torch.float64
    yield "dry_3d_37x23x19_f32", g3, wl.random_smooth_state(g3, 31), torch.float32
    gb, qb = wl.bubble_2d(96, 48)
    yield "bubble_2d_96x48_f64", gb, qb, torch.float64
    yield "bubble_2d_96x48_f32", gb, qb, torch.float32
    gj, qj = wl.jovian_3d(nx=24, ny=20, nz=40, mixture=True)
    yield "jovian_mixture_24x20x40_f32", gj, qj, torch.float32
    gk, qk, _ = wl.jovian_kessler_3d(nx=20, ny=18, nz=48, sediment=True)
    yield "jovian_sediment_20x18x48_f32", gk, qk, torch.float32
    gc, qc, _ = wl.convection_3d(256, 256, 128)
    yield "convection_256x256x128_f64", gc, qc, torch.float64
    yield "convection_256x256x128_f32", gc, qc, torch.float32


@pytest.mark.parametrize("case", list(cases()), ids=lambda c: c[0])
def test_device_dt_step_equals_host_dt_step(case):
    name, grid, q, dtype = case
    print(f"[rk3-cfl] {name}", flush=True)
    dg = snap.device_grid(grid, dtype=dtype)
    q0 = torch.as_tensor(q).to(dtype).cuda()
    host, dev = q0.clone(), q0.clone()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    cw = snap.workspace(dg, snap.SNAP_OP_CFL)
    wcfl = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    dt_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    for step in range(3):
        dt = snap.snap_cfl_dt(dg, host, CFL, cw)
        snap.snap_rk3_step(dg, host, dt, work)
        snap.snap_rk3_step_cfl(dg, dev, CFL, wcfl, dt_dev)
        torch.cuda.synchronize()
        got = float(dt_dev.item())
        assert got == dt, (step, got, dt)
        ih = grid.interior(host.cpu().numpy())
        idv = grid.interior(dev.cpu().numpy())
        assert np.array_equal(ih, idv), f"step {step}: device-dt step differs"
    assert np.isfinite(idv).all()


def test_device_dt_step_without_dt_output():
    grid, q = wl.bubble_2d(64, 32)
    dg = snap.device_grid(grid)
    a = torch.as_tensor(q).cuda()
    b = a.clone()
    w = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    snap.snap_rk3_step_cfl(dg, a, CFL, w)
    snap.snap_rk3_step_cfl(dg, b, CFL, w, torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert np.array_equal(grid.interior(a.cpu().numpy()), grid.interior(b.cpu().numpy()))


@pytest.mark.parametrize("case", list(cases()), ids=lambda c: c[0])
def test_multi_step_call_equals_single_steps(case):
    """snap_rk3_steps_cfl: four steps in one call; on 3-D grids without
    tracers each step's last stage reduces the next step's signal speed
    itself, and every dt and state must still equal the host's."""
    name, grid, q, dtype = case
    print(f"[rk3-cfl] steps {name}", flush=True)
    dg = snap.device_grid(grid, dtype=dtype)
    q0 = torch.as_tensor(q).to(dtype).cuda()
    host, dev = q0.clone(), q0.clone()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    cw = snap.workspace(dg, snap.SNAP_OP_CFL)
    n = 4
    dts = []
    for _ in range(n):
        dts.append(snap.snap_cfl_dt(dg, host, CFL, cw))
        snap.snap_rk3_step(dg, host, dts[-1], work)
    dt_dev = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    snap.snap_rk3_steps_cfl(dg, dev, CFL, n, snap.workspace(dg, snap.SNAP_OP_RK3_CFL), dt_dev)
    torch.cuda.synchronize()
    assert dt_dev.cpu().tolist() == dts
    assert np.array_equal(grid.interior(host.cpu().numpy()), grid.interior(dev.cpu().numpy()))


def state_cases():
    g3, _ = wl.dry_grid(37, 23, 19, 7400.0, 4600.0, 2850.0)
    yield "dry_3d_37x23x19_f64", g3, wl.random_smooth_state(g3, 41), torch.float64
    yield "dry_3d_37x23x19_f32", g3, wl.random_smooth_state(g3, 41), torch.float32
    gb, qb = wl.bubble_2d(96, 48)
    yield "bubble_2d_96x48_f64", gb, qb, torch.float64
    gt, _ = wl.dry_grid(21, 17, 15, 4200.0, 3400.0, 2250.0)
    gt.ntracer = 2
    yield "tracers_3d_21x17x15_f32", gt, wl.random_smooth_state(gt, 42), torch.float32
    gj, qj = wl.jovian_3d(nx=24, ny=20, nz=40, mixture=True)
    yield "jovian_mixture_24x20x40_f32", gj, qj, torch.float32


@pytest.mark.parametrize("case", list(state_cases()), ids=lambda c: c[0])
def test_state_flag_of_device_dt_steps(case):
    """A negative total energy planted on the host in one interior cell makes
    the CFL reduction NaN (no kernel branches on the data, so every kernel
    still runs to its end): snap_rk3_steps_status must report SNAP_E_STATE
    after the call, SNAP_OK for the same call on the clean state, and the
    flag must be cleared by the next call on the same workspace."""
    name, grid, q, dtype = case
    print(f"[rk3-cfl] state flag {name}", flush=True)
    dg = snap.device_grid(grid, dtype=dtype)
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    clean = torch.as_tensor(q).to(dtype).cuda()
    bad_host = q.copy()
    k, j, i = grid.nz // 2, grid.ny // 2, grid.nx // 3
    grid.interior(bad_host)[4, k, j, i] = -abs(grid.interior(bad_host)[4, k, j, i])
    bad = torch.as_tensor(bad_host).to(dtype).cuda()

    a = clean.clone()
    snap.snap_rk3_steps_cfl(dg, a, CFL, 3, work)
    snap.snap_rk3_steps_status(dg, work)
    assert torch.isfinite(grid.interior(a)).all()

    b = bad.clone()
    snap.snap_rk3_steps_cfl(dg, b, CFL, 3, work)
    with pytest.raises(snap.SnapError) as err:
        snap.snap_rk3_steps_status(dg, work)
    assert err.value.code == snap.SNAP_E_STATE
    assert not torch.isfinite(grid.interior(b)).all()

    # single-step entry point, then a clean call on the same workspace
    c = bad.clone()
    snap.snap_rk3_step_cfl(dg, c, CFL, work)
    with pytest.raises(snap.SnapError):
        snap.snap_rk3_steps_status(dg, work)
    d = clean.clone()
    snap.snap_rk3_step_cfl(dg, d, CFL, work)
    snap.snap_rk3_steps_status(dg, work)
