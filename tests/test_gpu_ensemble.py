"""GPU checks of the batched (ensemble) SSP-RK3 step.

* with the default tile shape (the one the single-domain kernel uses), every
  persistent-grid size gives, per member, bit for bit the state of separate
  snap_rk3_step calls; the other tile shapes run the same arithmetic but are
  separate template instances whose fused multiply-adds the compiler may form
  differently, so they agree within a few ulp (1e-14 FP64, 1e-6 FP32 relative
  to the field's largest magnitude);
* members match the FP64 oracle within the time-stepping bar of the parity
  tests;
* the autotuner returns an available variant and leaves the states untouched;
* members under the mixture equation of state (2-D, 1 to 4 tracers) and
  members with the HLLC flux (every tile variant without tracers) give, with
  the default tile shape, bit for bit the states of separate snap_rk3_step
  calls, and the other HLLC variants agree within the bars above; one member
  of each form matches the oracle after two steps;
* members that differ in equation of state or Riemann solver, and members
  with falling condensates, are rejected.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
from paper_1901_02955_amd import tuner
import workloads as wl
from tests import cases as C
from tests.test_gpu_parity import assert_steps_close, field_errors, rounding_sensitivity

pytestmark = pytest.mark.gpu

SIZES = ((20, 16), (37, 21), (16, 40), (64, 8), (3, 5))


def members(dtype=torch.float64, n=7, seed=4):
    ms = wl.ensemble_2d(n=n, seed=seed, sizes=SIZES)
    out = []
    for m, (g, q) in enumerate(ms):
        q = wl.random_smooth_state(g, 300 + m)   # all terms of the right-hand side active
        out.append((g, q))
    grids = [snap.device_grid(g, dtype=dtype) for g, _ in out]
    return out, grids


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_equals_separate_steps_bitwise(dtype):
    host, grids = members(dtype)
    dts = [0.15 + 0.01 * m for m in range(len(host))]
    ref = []
    for (g, q), dg, dt in zip(host, grids, dts):
        qd = torch.as_tensor(q).to(dtype).cuda()
        work = snap.workspace(dg, snap.SNAP_OP_RK3)
        for _ in range(2):
            snap.snap_rk3_step(dg, qd, dt, work)
        ref.append(qd)
    work = snap.batched_workspace(grids)
    for v, shape in tuner.candidates(grids):
        for nb in (0, 1, 5):
            print(f"[ensemble] {dtype} variant {v} {shape} nblocks {nb}", flush=True)
            qs = [torch.as_tensor(q).to(dtype).cuda() for _, q in host]
            for _ in range(2):
                snap.snap_rk3_step_batched(grids, qs, dts, work, v, nb)
            tol = 1e-14 if dtype == torch.float64 else 1e-6
            for m, (g, _) in enumerate(host):
                a = g.interior(qs[m].cpu().double().numpy())
                b = g.interior(ref[m].cpu().double().numpy())
                if v == 0:
                    assert np.array_equal(a, b), (v, nb, m)
                else:
                    for k in range(g.nvar):
                        scale = max(float(np.abs(b[k]).max()), 1e-300)
                        assert float(np.abs(a[k] - b[k]).max()) <= tol * scale, (v, nb, m, k)


def test_batched_members_match_oracle():
    host, grids = members(torch.float64, n=4)
    dts = [0.2, 0.15, 0.1, 0.12]
    qs = [torch.as_tensor(q).cuda() for _, q in host]
    work = snap.batched_workspace(grids)
    for _ in range(3):
        snap.snap_rk3_step_batched(grids, qs, dts, work)
    for m, (g, q) in enumerate(host):
        ref, kappa = rounding_sensitivity(g, q, dts[m], 3)
        assert_steps_close(g.interior(qs[m].cpu().numpy()), ref, kappa, f"member {m}")


def test_tuner_picks_available_variant(tmp_path, monkeypatch):
    monkeypatch.setenv("SNAP_TUNE_CACHE", str(tmp_path / "tune.json"))
    host, grids = members(torch.float32, n=5)
    qs = [torch.as_tensor(q).float().cuda() for _, q in host]
    before = [q.clone() for q in qs]
    res = tuner.tune_batched(grids, qs, [0.1] * len(qs), repeats=1)
    assert res["variant"] in [v for v, _ in tuner.candidates(grids)]
    assert all(torch.equal(a, b) for a, b in zip(qs, before))
    again = tuner.tune_batched(grids, qs, [0.1] * len(qs))
    assert again["variant"] == res["variant"]
    assert (tmp_path / "tune.json").exists()


def test_batched_rejects_mixed_members():
    host, grids = members(torch.float64, n=2)
    g3, _ = wl.dry_grid(8, 6, 5, 800.0, 600.0, 500.0)
    d3 = snap.device_grid(g3)
    with pytest.raises(snap.SnapError) as ei:
        snap.snap_batched_workspace_bytes([grids[0], d3])
    assert "3-D" in str(ei.value)
    f32 = snap.device_grid(host[1][0], dtype=torch.float32)
    with pytest.raises(snap.SnapError):
        snap.snap_batched_workspace_bytes([grids[0], f32])


def form_members(form, dtype):
    """2-D members of uneven sizes in smooth states: the mixture with 2
    tracers (a vapour and its cloud), or HLLC without tracers."""
    sizes = ((37, 21), (20, 16), (16, 40), (64, 8), (3, 5))
    out = []
    for m, (nx, nz) in enumerate(sizes):
        if form == "mixture":
            spec = dict(nx=nx, ny=1, nz=nz, nt=2, bc=(0, 0, 1), seed=500 + m, species=(0, 2))
            c = C.build_case(f"mix_member_{m}", spec)
            g = c.grid
        else:
            spec = dict(nx=nx, ny=1, nz=nz, nt=0, bc=(m % 2, 0, 1), seed=520 + m)
            c = C.build_case(f"hllc_member_{m}", spec)
            g = c.grid.copy(riemann=wl.RIEMANN_HLLC)
        out.append((g, c.q))
    return out, [snap.device_grid(g, dtype=dtype) for g, _ in out]


@pytest.mark.parametrize("form", ["mixture", "hllc"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_forms_equal_separate_steps(form, dtype):
    host, grids = form_members(form, dtype)
    dts = [0.1 + 0.01 * m for m in range(len(host))]
    ref = []
    for (g, q), dg, dt in zip(host, grids, dts):
        qd = torch.as_tensor(q).to(dtype).cuda()
        work = snap.workspace(dg, snap.SNAP_OP_RK3)
        for _ in range(2):
            snap.snap_rk3_step(dg, qd, dt, work)
        ref.append(qd)
    work = snap.batched_workspace(grids)
    for v, shape in tuner.candidates(grids):
        print(f"[ensemble] {form} {dtype} variant {v} {shape}", flush=True)
        qs = [torch.as_tensor(q).to(dtype).cuda() for _, q in host]
        for _ in range(2):
            snap.snap_rk3_step_batched(grids, qs, dts, work, v)
        tol = 1e-14 if dtype == torch.float64 else 1e-6
        for m, (g, _) in enumerate(host):
            a = g.interior(qs[m].cpu().double().numpy())
            b = g.interior(ref[m].cpu().double().numpy())
            if v == 0:
                assert np.array_equal(a, b), (form, v, m)
            else:
                errs = field_errors(a, b)
                assert all(e <= tol for e in errs), (form, v, m, errs)


@pytest.mark.parametrize("form", ["mixture", "hllc"])
def test_batched_forms_match_oracle(form):
    host, grids = form_members(form, torch.float64)
    dts = [0.1 + 0.01 * m for m in range(len(host))]
    qs = [torch.as_tensor(q).cuda() for _, q in host]
    work = snap.batched_workspace(grids)
    for _ in range(2):
        snap.snap_rk3_step_batched(grids, qs, dts, work)
    for m in (0, 2):
        g, q = host[m]
        ref, kappa = rounding_sensitivity(g, q, dts[m], 2)
        assert_steps_close(g.interior(qs[m].cpu().numpy()), ref, kappa, f"{form} member {m}")


def test_batched_rejects_mixed_forms():
    mix, gm = form_members("mixture", torch.float64)
    hl, gh = form_members("hllc", torch.float64)
    plain = snap.device_grid(hl[0][0].copy(riemann=wl.RIEMANN_LMARS))
    with pytest.raises(snap.SnapError):
        snap.snap_batched_workspace_bytes([gh[0], plain])
    g0 = mix[0][0]
    g_passive = snap.device_grid(g0.copy(eos=wl.EOS_PASSIVE))
    with pytest.raises(snap.SnapError):
        snap.snap_batched_workspace_bytes([gm[0], g_passive])
