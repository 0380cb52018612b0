#!/usr/bin/env python3
"""Throughput of the WENO5 + LMARS SSP-RK3 step on one MI355X.

Workload: 3-D dry convection, 256 x 256 x 128 cells (20 x 20 x 10 km), five
conserved variables, isentropic 300 K hydrostatic base state, seeded uniform
theta noise of +-0.1 K in the lowest 10 levels, periodic in x and y, rigid
lids in z, CFL 0.9. One timed step = one three-stage SSP-RK3 step whose time
step dt = CFL / (maximum signal speed of Q^n) is formed on the device: three
fused stage kernels that read the ghost cells at their sources (no fills),
the last of which also reduces the next step's signal speed. The state lives
in HBM before the timed region starts. `value` is the median of 5 timed
calls of `--steps` steps each; the stage kernel's launch time comes from a
separate pass with hipEvents around every stage launch.

The FP64 path is the headline (`value`); the FP32 form (FP32 storage and
stencil arithmetic, FP64 reference state and E -> p inversion) runs on the
same workload and is reported under `variants.f32`.

Roofline of the dominant kernel (the fused stage kernel), from its average
launch duration:
* `roofline` (bound "alu": the measured HBM traffic is far below the memory
  roofline, the kernel is limited by vector-ALU issue): algorithmic flops per
  launch = algorithmic_flops_per_cell_stage() x cells, against the MI355X
  vector peak of the element type;
* `hbm_roofline`: algorithmic HBM bytes per launch = (8/3) * nvar *
  sizeof(element) * cells (stage 1 reads Q and writes Q1, stages 2 and 3 read
  Q_s and Q^n and write the next state: 8 state passes per step, averaged over
  the three launches), against 8 TB/s.

CPU baseline: the FP64 oracle (PyTorch CPU, all host threads of this process)
on a bounded sample of the same workload: SSP-RK3 steps (4 to 24, about 15 s)
of a 128 x 128 x 128 column block cut from the same initial state (periodic in
x and y); `cpu_oracle_sections` times it on samples of the other workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s of WENO5+LMARS RK3 step (FP32 vs FP64), % HBM roofline"
HBM_PEAK_GBS = 8000.0
NX, NY, NZ = 256, 256, 128
CFL = 0.9


FP64_PEAK_TFLOPS = 78.6     # MI355X vector FP64 (FMA = 2 flops)
FP32_PEAK_TFLOPS = 157.3    # MI355X vector FP32 (counts packed FP32, which this build does not emit)


def algorithmic_flops_per_cell_stage(ntracer: int, ndir: int, mixture: bool = False,
                                     hllc: bool = False) -> int:
    """Floating-point operations of one right-hand side + stage update of one cell.

    Counted from the method's formulas (+, -, *, /, sqrt = 1 flop each, a fused
    multiply-add = 2), with no halo redundancy, address arithmetic or data
    movement: conserved -> primitive 14 + NT; WENO5 per variable and direction
    (both faces of the cell, shared smoothness indicators) 78; LMARS per face
    37 + NT; divergence 3 per variable and direction; gravity 4; Runge-Kutta
    combination 4 per variable averaged over the three stages. The mixture
    equation of state adds 6 NT + 2 to conserved -> primitive (chemical
    energy, the two weighted sums, their ratio) and 12 NT + 10 per face (the
    sums of both sides, their effective gamma and internal energy). HLLC in
    place of LMARS costs 66 + 3 NT per face: the two sound speeds and Davis
    bounds 10, the contact speed 11, the upwind side's physical flux 14 + NT,
    its star-state correction 31 + 2 NT.
    """
    nv = 5 + ntracer
    face = (66 + 3 * ntracer) if hllc else (37 + ntracer)
    n = (14 + ntracer) + ndir * nv * 78 + ndir * face + ndir * 3 * nv + 4 + 4 * nv
    if mixture and ntracer > 0:
        n += 6 * ntracer + 2 + ndir * (12 * ntracer + 10)
    return n


# Signal-speed sum of one cell, the CFL quantity sum_d (|u_d| + c) / dx_d:
# 1 / rho 1, velocities 3, kinetic energy 6, pressure 2, gamma p / rho 2,
# square root 1, three (|u_d| + c) * (1 / dx_d) 6, their sum 2.
CFL_FLOPS_PER_CELL = 23


# sources the stage kernel and its launch (tiling, z-chunks) are built from, with
# build.py's flags
STAGE_SOURCES = ("snap_device.h", "snap_stage.h", "snap_internal.h", "stage_launch.h",
                 "stage_dry_f64.hip", "stage_dry_f32.hip", "stage_f64.hip", "stage_f32.hip",
                 "snap_api.hip")


def stage_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1901_02955_amd", "csrc")
    for name in STAGE_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    # the compiler flags, which differ between the stage files
    with open(os.path.join(ROOT, "paper_1901_02955_amd", "build.py"), "rb") as f:
        h.update(b"build.py")
        h.update(f.read())
    return h.hexdigest()[:16]


def _profile_value(key: str):
    """A value of the committed counter summary of the stage kernel.

    Returns None unless the counters were taken on the current kernel sources.
    """
    path = os.path.join(ROOT, "profiles", "stage_kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("sources_digest") != stage_sources_digest():
        return None
    return float(vals[key]) if key in vals else None


def measured_traffic(dtype_name: str):
    """HBM bytes per stage launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs."""
    return _profile_value(f"bytes_per_launch_{dtype_name}")


def _timed(fn, repeats: int):
    """Wall-clock seconds of ``repeats`` calls of fn, each bracketed by device syncs."""
    import torch

    out = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return out


def _stage_pass(fn):
    """Average stage-kernel launch time (s) and launch count of one call of fn,
    from hipEvents recorded around every stage launch on its stream."""
    import torch

    import paper_1901_02955_amd as snap

    torch.cuda.synchronize()
    snap.snap_stage_timing_enable(True)
    fn()
    torch.cuda.synchronize()
    ms, n = snap.snap_stage_timing_read()
    snap.snap_stage_timing_enable(False)
    return ms / 1e3 / max(n, 1), n


def run_gpu(dtype, steps: int, warmup: int, hllc: bool = False, repeats: int = 5,
            perturbation: bool = False):
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q, _ = wl.convection_3d(NX, NY, NZ)
    if hllc:
        grid = grid.copy(riemann=wl.RIEMANN_HLLC)
    if perturbation:
        q = wl.to_perturbation(grid, q)
    dg = snap.device_grid(grid, dtype=dtype, storage=snap.SNAP_STORE_PERTURBATION if perturbation
                          else snap.SNAP_STORE_TOTAL)
    qd = torch.as_tensor(q).to(dtype).cuda().contiguous()
    del q
    # each step takes dt = CFL / (maximum signal speed of Q^n) on the device
    # (snap_rk3_steps_cfl: the stages read dt from device memory, and the last
    # stage of a step reduces the next step's signal speed), so the steps run
    # back to back without a host round trip
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    dt_dev = torch.zeros(max(steps, warmup, 1), dtype=torch.float64, device="cuda")
    if warmup > 0:
        snap.snap_rk3_steps_cfl(dg, qd, CFL, warmup, work, dt_dev)

    def call():
        snap.snap_rk3_steps_cfl(dg, qd, CFL, steps, work, dt_dev)

    # the timed windows carry no instrumentation; the stage kernel's launch
    # time comes from a separate pass of the same call with hipEvents
    times = _timed(call, repeats)
    snap.snap_rk3_steps_status(dg, work)
    elapsed = _median(times)
    dt = float(dt_dev[steps - 1].item())
    avg_launch_s, launches = _stage_pass(call)
    cells = NX * NY * NZ
    esize = 8 if dtype == torch.float64 else 4
    nvar = dg.nvar
    bytes_per_launch = 8.0 / 3.0 * nvar * esize * cells
    # the last stage of every timed step also reduces the signal speed of the
    # state it writes (3-D, no tracers: the next step's time step, and the
    # state check after the call's last step): its flops count, per launch
    fused_share = 1.0 / 3.0
    flops_per_launch = (algorithmic_flops_per_cell_stage(dg.ntracer, 3, hllc=hllc)
                        + CFL_FLOPS_PER_CELL * fused_share) * cells
    gbs = bytes_per_launch / avg_launch_s / 1e9
    tflops = flops_per_launch / avg_launch_s / 1e12
    name = "f64" if dtype == torch.float64 else "f32"
    peak = FP64_PEAK_TFLOPS if name == "f64" else FP32_PEAK_TFLOPS
    traffic = None if (hllc or perturbation) else measured_traffic(name)
    res = {
        "value": cells * steps / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "repeats": repeats,
        "spread": _spread(times),
        "stage_kernel_avg_ms": avg_launch_s * 1e3,
        "stage_launches": launches,
        "roofline": {
            "bound": "alu", "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
            "frac": tflops / peak, "traffic": traffic,
        },
        "hbm_roofline": {
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "measured_bytes_per_launch": traffic,
            "measured_frac": (traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
        },
        # VALU instructions issued / (256 CUs x one wave instruction per cycle x
        # active cycles), from the committed SQ_INSTS_VALU / GRBM_GUI_ACTIVE run
        "valu_utilisation": None if (hllc or perturbation) else _profile_value(f"valu_issue_util_{name}"),
        "final_dt": dt,
    }
    del qd, work, dt_dev
    torch.cuda.empty_cache()
    return res


def run_jovian(steps: int, warmup: int, mixture: bool = False, repeats: int = 5):
    """3-D Jovian-like column 512x512x256, FP32, 4 tracer densities (vapours and
    clouds); passive, or under the mixture equation of state."""
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q = wl.jovian_3d(mixture=mixture)
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = torch.as_tensor(q).float().cuda().contiguous()
    del q
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    if warmup > 0:
        snap.snap_rk3_steps_cfl(dg, qd, CFL, warmup, work)

    def call():
        snap.snap_rk3_steps_cfl(dg, qd, CFL, steps, work)

    times = _timed(call, repeats)
    snap.snap_rk3_steps_status(dg, work)
    el = _median(times)
    avg_s, _ = _stage_pass(call)
    cells = grid.nx * grid.ny * grid.nz
    avg = avg_s
    flops = algorithmic_flops_per_cell_stage(4, 3, mixture) * cells
    byts = 8.0 / 3.0 * 9 * 4 * cells
    eos = ("mixture equation of state (water and ammonia vapours and clouds)" if mixture
           else "passive tracers")
    out = {"workload": "3-D Jovian-like column 512x512x256 (5.5 km x 5.5 km x 1.5625 km), FP32, "
                       f"5 conserved + 4 tracer densities, {eos}, CFL 0.9",
           "value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el / steps * 1e3,
           "steps": steps, "repeats": repeats, "spread": _spread(times),
           "stage_kernel_avg_ms": avg * 1e3,
           "alu_frac": flops / avg / 1e12 / FP32_PEAK_TFLOPS,
           "hbm_frac_algorithmic": byts / avg / 1e9 / HBM_PEAK_GBS}
    del qd, work
    torch.cuda.empty_cache()
    return out


def run_jovian_kessler(steps: int, warmup: int, sediment: bool = True, repeats: int = 5):
    """The Jovian-like column with water and ammonia vapour, cloud and
    precipitation (6 tracers) under the mixture equation of state, FP32: an
    SSP-RK3 step (with the precipitation falling at 8 and 5 m/s if
    ``sediment``) followed by a Kessler microphysics step of the same dt."""
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q, kes = wl.jovian_kessler_3d(sediment=sediment)
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = torch.as_tensor(q).float().cuda().contiguous()
    del q
    params = snap.kessler_params(kes)
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    cw = snap.workspace(dg, snap.SNAP_OP_CFL)

    def step():
        dt = snap.snap_cfl_dt(dg, qd, CFL, cw)
        snap.snap_rk3_step(dg, qd, dt, work)
        snap.snap_kessler_step(dg, qd, dt, params)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the microphysics kernel alone, on the stream, over the same number of calls
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        snap.snap_kessler_step(dg, qd, 1e-9, params)
    e1.record()
    torch.cuda.synchronize()
    micro_ms = e0.elapsed_time(e1) / steps
    # the microphysics adjoint (J^T of the Kessler step in place on a seeded
    # cotangent), on the stream, over the same number of calls and a CFL dt
    dt_adj = snap.snap_cfl_dt(dg, qd, CFL, cw)
    qbar = torch.randn(dg.interior_shape, dtype=torch.float32, device="cuda",
                       generator=torch.Generator(device="cuda").manual_seed(17))
    snap.snap_kessler_step_adjoint(dg, qd, dt_adj, params, qbar)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        snap.snap_kessler_step_adjoint(dg, qd, dt_adj, params, qbar)
    e1.record()
    torch.cuda.synchronize()
    micro_adj_ms = e0.elapsed_time(e1) / steps
    del qbar

    def steps_fn():
        for _ in range(steps):
            step()

    times = _timed(steps_fn, repeats)
    el = _median(times)
    cells = grid.nx * grid.ny * grid.nz
    byts = (11 + 6) * 4 * cells          # reads every field, writes the six tracers
    fall = "falling precipitation (8 and 5 m/s), " if sediment else ""
    out = {"workload": "3-D Jovian-like column 512x512x256, FP32, water and ammonia vapour, cloud and "
                       f"precipitation (6 tracers), {fall}mixture equation of state, SSP-RK3 step + "
                       "Kessler microphysics step, CFL 0.9",
           "value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el / steps * 1e3,
           "steps": steps, "repeats": repeats, "spread": _spread(times), "microphysics_ms": micro_ms,
           "microphysics_hbm_frac": byts / (micro_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "microphysics_share": micro_ms / (el / steps * 1e3),
           "microphysics_adjoint_ms": micro_adj_ms}
    del qd, work, cw
    torch.cuda.empty_cache()
    return out


def run_jovian_satadj(steps: int, warmup: int, repeats: int = 5):
    """The Jovian-like column with water and ammonia vapour and cloud (4
    tracers) under the mixture equation of state, FP32: an SSP-RK3 step
    followed by saturation adjustment (App. D)."""
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q, adj = wl.jovian_satadj_3d()
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = torch.as_tensor(q).float().cuda().contiguous()
    del q
    params = snap.satadj_params(adj)
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    # the adjustment alone, each call on a fresh copy of the initial state
    # (supersaturated aloft, clouds seeded): a second call on an adjusted
    # state would stop after one sweep
    q0 = qd.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    adj_ms = 0.0
    for r in range(steps + 1):
        qd.copy_(q0)
        torch.cuda.synchronize()
        e0.record()
        snap.snap_saturation_adjust(dg, qd, params)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            adj_ms += e0.elapsed_time(e1)
    adj_ms /= steps
    # its adjoint (J^T in place on a seeded cotangent) from the same initial state
    qbar = torch.randn(dg.interior_shape, dtype=torch.float32, device="cuda",
                       generator=torch.Generator(device="cuda").manual_seed(19))
    snap.snap_saturation_adjust_adjoint(dg, q0, params, qbar)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        snap.snap_saturation_adjust_adjoint(dg, q0, params, qbar)
    e1.record()
    torch.cuda.synchronize()
    adj_adjoint_ms = e0.elapsed_time(e1) / steps
    del q0, qbar

    def step():
        snap.snap_rk3_step_cfl(dg, qd, CFL, work)
        snap.snap_saturation_adjust(dg, qd, params)

    for _ in range(warmup):
        step()

    def steps_fn():
        for _ in range(steps):
            step()

    times = _timed(steps_fn, repeats)
    snap.snap_rk3_steps_status(dg, work)
    el = _median(times)
    cells = grid.nx * grid.ny * grid.nz
    byts = (9 + 4) * 4 * cells          # reads every field, writes the four tracers
    out = {"workload": "3-D Jovian-like column 512x512x256, FP32, water and ammonia vapour and cloud "
                       "(4 tracers), mixture equation of state, SSP-RK3 step + saturation "
                       "adjustment, CFL 0.9",
           "value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el / steps * 1e3,
           "steps": steps, "repeats": repeats, "spread": _spread(times), "adjustment_ms": adj_ms,
           "adjustment_hbm_frac": byts / (adj_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "adjustment_share": adj_ms / (el / steps * 1e3), "adjustment_adjoint_ms": adj_adjoint_ms}
    del qd, work
    torch.cuda.empty_cache()
    return out


def run_ensemble(steps: int, repeats: int = 5):
    """64 uneven 2-D bubbles (FP32): one persistent launch per stage vs separate steps."""
    import torch

    import paper_1901_02955_amd as snap
    from paper_1901_02955_amd import tuner
    import workloads as wl

    members = wl.ensemble_2d(64, seed=4)
    grids = [snap.device_grid(g, dtype=torch.float32) for g, _ in members]
    qs = [torch.as_tensor(q).float().cuda().contiguous() for _, q in members]
    cw = snap.workspace(grids[0], snap.SNAP_OP_CFL)
    dts = [snap.snap_cfl_dt(g, q, CFL, cw) for g, q in zip(grids, qs)]
    cells = sum(g.nx * g.nz for g in grids)
    tuned = tuner.tune_batched(grids, qs, dts, repeats=3, use_cache=False)
    bw = snap.batched_workspace(grids)
    work = [snap.workspace(g, snap.SNAP_OP_RK3) for g in grids]

    def timed(fn):
        fn()

        def steps_fn():
            for _ in range(steps):
                fn()

        return _median(_timed(steps_fn, repeats))

    def batched():
        snap.snap_rk3_step_batched(grids, qs, dts, bw, tuned["variant"], tuned["nblocks"])

    def separate():
        for g, q, dt, w in zip(grids, qs, dts, work):
            snap.snap_rk3_step(g, q, dt, w)

    tb, ts = timed(batched), timed(separate)
    return {"workload": "64 uneven 2-D dry bubbles (128x128 .. 512x256, seeded), FP32, "
                        "per-member CFL 0.9 time step",
            "members": len(grids), "cells": cells, "steps": steps, "repeats": repeats,
            "batched_value": cells * steps / tb, "separate_value": cells * steps / ts,
            "unit": "cell-updates/s", "batched_ms_per_step": tb / steps * 1e3,
            "separate_ms_per_step": ts / steps * 1e3, "speedup": ts / tb,
            "launches_per_step": {"batched": 6, "separate": 6 * len(grids)},
            "tuned": {k: tuned[k] for k in ("variant", "tile", "nblocks")}}


def _median(xs):
    s = sorted(xs)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def _spread(xs):
    """(max - min) / median of repeated timings."""
    m = _median(xs)
    return (max(xs) - min(xs)) / m if m > 0 else None


def top_kinetic_energy(grid, q, levels=16):
    """Kinetic energy (J) of the top ``levels`` levels of a padded state, summed in FP64."""
    g0 = grid.gy if grid.ny > 1 else 0
    G0 = 3
    top = q[:, G0 + grid.nz - levels:G0 + grid.nz, g0:g0 + grid.ny, G0:G0 + grid.nx].double()
    dv = grid.dx * grid.dy * grid.dz
    return 0.5 * dv * ((top[1] ** 2 + top[2] ** 2 + top[3] ** 2) / top[0]).sum()


def gradient_check(nx, ny, nz, nsteps, every, seeds, h=1e-4, lx=None, ly=None, lz=None,
                   repeats=0):
    """Gradient of the top-level kinetic energy with respect to the initial theta' field.

    The state is built from theta' (and the seeded top-level flow) by
    ``workloads.state_from_theta`` in torch, so autograd carries the gradient of
    the checkpointed RK3 run (``rk3_run``: the library's RK3 adjoint) back to
    theta'. The same gradient is taken in FP32 (the workload's form) and in FP64,
    the FP32 one with and without kept stage states (bit-identical), and each is
    compared with central differences of the FP64 forward along seeded theta'
    directions (standard normal per cell, in K), Richardson-extrapolated from
    steps h and h / 2. dt is the CFL 0.9 step of the initial state, held fixed.
    With ``repeats`` > 0 the FP32 forward alone and the FP32 forward with
    checkpoints + backward are timed that many times (medians reported).
    """
    import numpy as np
    import torch

    import paper_1901_02955_amd as snap
    from paper_1901_02955_amd.autograd import rk3_run
    import workloads as wl

    kw = {}
    if lx is not None:
        kw = dict(lx=lx, ly=ly, lz=lz)
    grid, base, dth, vel, dp = wl.convection_flow_3d(nx, ny, nz, **kw)
    th0 = torch.as_tensor(dth, device="cuda")
    vd = torch.as_tensor(vel, device="cuda")
    pd = torch.as_tensor(dp, device="cuda")
    dg = {torch.float64: snap.device_grid(grid, dtype=torch.float64),
          torch.float32: snap.device_grid(grid, dtype=torch.float32)}
    dg_p32 = snap.device_grid(grid, dtype=torch.float32, storage=snap.SNAP_STORE_PERTURBATION)
    with torch.no_grad():
        q64 = wl.state_from_theta(grid, base, th0, vd, pd)
    dt = snap.snap_cfl_dt(dg[torch.float64], q64, CFL, snap.workspace(dg[torch.float64], snap.SNAP_OP_CFL))
    del q64

    def ad_gradient(dtype, keep=True, perturbation=False):
        th = th0.clone().requires_grad_(True)
        q0 = wl.state_from_theta(grid, base, th, vd, pd)
        if perturbation:
            # the state stored as rho - rhobar and E - pbar / (gamma - 1)
            out = rk3_run(dg_p32, wl.to_perturbation(grid, q0).to(dtype), dt, nsteps, every)
            out = wl.from_perturbation(grid, out.double())
        else:
            out = rk3_run(dg[dtype], q0.to(dtype), dt, nsteps, every, keep_stages=keep)
        L = top_kinetic_energy(grid, out)
        L.backward()
        return th.grad.detach(), float(L.detach())

    res = {}
    if repeats > 0:
        work = snap.workspace(dg[torch.float32], snap.SNAP_OP_RK3)
        with torch.no_grad():
            q32 = wl.state_from_theta(grid, base, th0, vd, pd).float()
        fwd, bwd, fck = [], [], []
        for _ in range(repeats):
            qf = q32.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nsteps):
                snap.snap_rk3_step(dg[torch.float32], qf, dt, work)
            torch.cuda.synchronize()
            fwd.append(time.perf_counter() - t0)
            x = q32.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = rk3_run(dg[torch.float32], x, dt, nsteps, every)
            L = top_kinetic_energy(grid, out)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fck.append(t1 - t0)
            bwd.append(t2 - t1)
            del x, out, qf
        del work, q32
        res.update({"forward_s": _median(fwd), "forward_spread": _spread(fwd),
                    "forward_with_checkpoints_s": _median(fck), "backward_s": _median(bwd),
                    "backward_spread": _spread(bwd), "repeats": repeats,
                    "adjoint_forward_ratio": _median(bwd) / _median(fwd)})
    g32, L32 = ad_gradient(torch.float32)
    g32_re, _ = ad_gradient(torch.float32, keep=False)
    kept_bitwise = bool(torch.equal(g32, g32_re))
    del g32_re
    g32p, _ = ad_gradient(torch.float32, perturbation=True)
    g64, L64 = ad_gradient(torch.float64)
    torch.cuda.empty_cache()

    work64 = snap.workspace(dg[torch.float64], snap.SNAP_OP_RK3)

    def loss64(th):
        with torch.no_grad():
            q = wl.state_from_theta(grid, base, th, vd, pd)
            for _ in range(nsteps):
                snap.snap_rk3_step(dg[torch.float64], q, dt, work64)
            return float(top_kinetic_energy(grid, q))

    rows = []
    for s in seeds:
        d = torch.as_tensor(wl.seeded_normal((nz, ny, nx), s), device="cuda")

        def central(hh):
            return (loss64(th0 + hh * d) - loss64(th0 - hh * d)) / (2.0 * hh)

        fd = (4.0 * central(0.5 * h) - central(h)) / 3.0
        a64 = float((g64 * d).sum())
        a32 = float((g32.double() * d).sum())
        a32p = float((g32p.double() * d).sum())
        rows.append((s, fd, a64, a32, a32p))
        print(f"[gradient] seed {s}: FD {fd:.10e}  AD64 {a64:.10e}  AD32 {a32:.10e}  "
              f"AD32 perturbation storage {a32p:.10e}", flush=True)
    fd = np.array([r[1] for r in rows])
    a64 = np.array([r[2] for r in rows])
    a32 = np.array([r[3] for r in rows])
    a32p = np.array([r[4] for r in rows])
    # <grad J, delta> with delta standard normal per cell has the spread
    # |grad J|; the differences are measured against that scale (the RMS of the
    # 32 differences) and, separately, against each direction's own value
    rms = float(np.sqrt(np.mean(fd ** 2)))
    res.update({
        "dt": dt, "loss_fp64": L64, "loss_fp32": L32,
        "grad_norm_fp32": float(g32.double().norm()), "grad_norm_fp64": float(g64.norm()),
        "grad_rel_l2_fp32_vs_fp64": float((g32.double() - g64).norm() / g64.norm()),
        "kept_vs_recomputed_stages_bitwise": kept_bitwise,
        "fd_directions": len(rows), "fd_seeds": [int(seeds[0]), int(seeds[-1])], "fd_h_kelvin": h,
        "fd_rms": rms,
        "fp64_adjoint": {"max_err_over_rms": float(np.max(np.abs(a64 - fd)) / rms),
                         "max_err_rel_own": float(np.max(np.abs(a64 - fd) / np.abs(fd)))},
        "fp32_adjoint": {"max_err_over_rms": float(np.max(np.abs(a32 - fd)) / rms),
                         "median_err_over_rms": float(np.median(np.abs(a32 - fd)) / rms),
                         "max_err_rel_own": float(np.max(np.abs(a32 - fd) / np.abs(fd)))},
        "fp32_perturbation_storage_adjoint": {
            "max_err_over_rms": float(np.max(np.abs(a32p - fd)) / rms),
            "median_err_over_rms": float(np.median(np.abs(a32p - fd)) / rms),
            "grad_rel_l2_vs_fp64": float((g32p.double() - g64).norm() / g64.norm())},
    })
    return res


# Bars of the gradient check: largest |<grad J, delta> - central difference|
# over the 32 directions, relative to the RMS of the differences. The FP64
# adjoint is the exact reverse of the FP64 forward; what remains is the
# differences' own error, of order h where a difference straddles a switch of
# LMARS's upwind side (measured 3e-5 at h = 1e-4 K, 2.5e-4 at 1e-3 K). The FP32
# adjoint differentiates the FP32 trajectory, whose vertical momentum is about
# 1 % off the FP64 one after 200 steps (FP32 storage of E), and its gradient is
# as far off the FP64 one (measured 1.1 % in the L2 norm, 2.2 % at most along
# a direction).
GRAD_TOL_FP64 = 3e-4
GRAD_TOL_FP32 = 5e-2


def run_adjoint(nsteps: int = 200, every: int = 20, ndir: int = 32, repeats: int = 5):
    """The gradient workload at its own size: 256x256x128, FP32, 200 SSP-RK3 steps
    with a checkpoint every 20, loss = kinetic energy of the top 16 levels,
    gradient with respect to the initial theta' field, checked against FP64
    central differences on 32 seeded directions (seeds 5-36); adjoint / forward
    time ratio (medians of ``repeats`` timings)."""
    res = gradient_check(NX, NY, NZ, nsteps, every, list(range(5, 5 + ndir)), repeats=repeats)
    res["within_tolerance"] = bool(res["fp64_adjoint"]["max_err_over_rms"] <= GRAD_TOL_FP64 and
                                   res["fp32_adjoint"]["max_err_over_rms"] <= GRAD_TOL_FP32)
    res["tolerance"] = {"fp64_adjoint": GRAD_TOL_FP64, "fp32_adjoint": GRAD_TOL_FP32}
    res = {"workload": "3-D dry convection 256x256x128 (theta' noise in the lowest 10 levels) with "
                       "a seeded smooth flow in the top 16 levels and a smooth 30 Pa pressure "
                       "perturbation, FP32, 200 SSP-RK3 steps of the initial CFL 0.9 dt, checkpoint "
                       "every 20, loss = kinetic energy of the top 16 levels, gradient w.r.t. the "
                       "initial theta' field; checked against FP64 central differences (Richardson, "
                       "h = 1e-4 K) on 32 seeded directions", **res}
    return res


def run_fp32_error(steps: int = 100, checkpoints=(25, 50, 75, 100)):
    """Per-field error of the FP32 form against FP64 after 100 steps, and its cause.

    Every run starts from the same state, the 256x256x128 convection state
    rounded to FP32, and takes the same fixed time step (the CFL 0.9 step of
    that state), so input rounding does not enter the comparison. The
    reference is the FP64 path (which matches the CPU oracle within 1e-12 per
    field on the parity cases and on sampled blocks of this grid). Errors are
    given relative to max|field| and relative to max|field - base|, the
    deviation from the hydrostatic base state (rho_bar_k, zero momentum,
    p_bar_k / (gamma - 1)), which is what the flow has developed.

    Attribution: two more runs take every stage in FP64 arithmetic (three
    snap_rhs calls per step in FP64, the stage combination in FP64) but round
    the stored stage states to FP32, all fields or E alone. If FP32 storage of
    E explains the error of the FP32 form, the E-only run shows errors of the
    same size.
    """
    import numpy as np
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q, _ = wl.convection_3d(NX, NY, NZ)
    q32 = q.astype(np.float32).astype(np.float64)
    del q
    G0 = 3
    nz = grid.nz
    base = np.zeros(grid.interior_shape)
    base[0] = grid.rhobar_cell[G0:G0 + nz][:, None, None]
    base[4] = grid.pbar_cell[G0:G0 + nz][:, None, None] / (grid.gamma - 1.0)
    dg64 = snap.device_grid(grid, dtype=torch.float64)
    dg32 = snap.device_grid(grid, dtype=torch.float32)
    q0 = torch.as_tensor(q32).cuda()
    dt = snap.snap_cfl_dt(dg64, q0, CFL, snap.workspace(dg64, snap.SNAP_OP_CFL))

    def interior_np(qd):
        return grid.interior(qd.double().cpu().numpy()).copy()

    def run_path(dtype):
        dg = dg64 if dtype == torch.float64 else dg32
        qd = q0.to(dtype).clone()
        work = snap.workspace(dg, snap.SNAP_OP_RK3)
        snaps = {}
        for n in range(1, steps + 1):
            snap.snap_rk3_step(dg, qd, dt, work)
            if n in checkpoints:
                snaps[n] = interior_np(qd)
        return snaps

    def run_rounded(fields):
        # FP64 stages with the stored stage states rounded to FP32 in `fields`
        qd = q0.clone()
        rhs = torch.empty(dg64.interior_shape, dtype=torch.float64, device="cuda")
        gy = grid.gy

        def inner(x):
            return x[:, G0:G0 + nz, gy:gy + grid.ny, G0:G0 + grid.nx]

        def rnd(x):
            i = inner(x)
            i[fields] = i[fields].float().double()
            return x

        snaps = {}
        for n in range(1, steps + 1):
            snap.snap_rhs(dg64, qd, rhs)
            q1 = qd.clone()
            inner(q1).add_(rhs, alpha=dt)
            rnd(q1)
            snap.snap_rhs(dg64, q1, rhs)
            q2 = q1.clone()
            inner(q2).add_(rhs, alpha=dt)
            inner(q2).mul_(0.25).add_(inner(qd), alpha=0.75)
            rnd(q2)
            snap.snap_rhs(dg64, q2, rhs)
            inner(q2).add_(rhs, alpha=dt)
            inner(qd).mul_(1.0 / 3.0).add_(inner(q2), alpha=2.0 / 3.0)
            rnd(qd)
            del q1, q2
            if n in checkpoints:
                snaps[n] = interior_np(qd)
        return snaps

    ref = run_path(torch.float64)
    f32 = run_path(torch.float32)
    all32 = run_rounded(slice(0, 5))
    e32 = run_rounded(slice(4, 5))
    names = ["rho", "rho_u", "rho_v", "rho_w", "E"]

    def table(got, b):
        out = {}
        for v, name in enumerate(names):
            d = got[v] - b[v]
            dev = b[v] - base[v]
            out[name] = {"max_rel": float(np.abs(d).max() / np.abs(b[v]).max()),
                         "l2_rel": float(np.sqrt((d ** 2).mean() / (b[v] ** 2).mean())),
                         "max_rel_dev": float(np.abs(d).max() / np.abs(dev).max()),
                         "l2_rel_dev": float(np.sqrt((d ** 2).mean() / (dev ** 2).mean()))}
        return out

    fields = table(f32[steps], ref[steps])
    history = {str(n): {name: fields_n[name]["max_rel_dev"] for name in names}
               for n, fields_n in ((n, table(f32[n], ref[n])) for n in checkpoints)}
    attribution = {"fp64_arithmetic_fp32_storage_all": table(all32[steps], ref[steps]),
                   "fp64_arithmetic_fp32_storage_E_only": table(e32[steps], ref[steps])}
    del q0, ref, f32, all32, e32

    # the FP32 form with perturbation storage (rho - rhobar, E - pbar / (gamma - 1)),
    # from its own FP32 rounding, against FP64 steps from that same state
    _, qfull, _ = wl.convection_3d(NX, NY, NZ)
    p32 = wl.to_perturbation(grid, qfull).astype(np.float32)
    del qfull
    start = wl.from_perturbation(grid, p32.astype(np.float64))
    dgp = snap.device_grid(grid, dtype=torch.float32, storage=snap.SNAP_STORE_PERTURBATION)
    q0 = torch.as_tensor(start).cuda()
    refp = run_path(torch.float64)
    qp = torch.as_tensor(p32).cuda()
    wp = snap.workspace(dgp, snap.SNAP_OP_RK3)
    for _ in range(steps):
        snap.snap_rk3_step(dgp, qp, dt, wp)
    gotp = grid.interior(wl.from_perturbation(grid, qp.double().cpu().numpy()))
    fields_p = table(gotp, refp[steps])
    del q0, qp, wp, refp, p32, start
    torch.cuda.empty_cache()
    return {"workload": f"3-D dry convection 256x256x128 (state rounded to FP32 for every run), "
                        f"{steps} steps of fixed dt = {dt:.6g} s; reference: the FP64 path",
            "fields": fields, "max_rel_dev_by_step": history, "attribution": attribution,
            "fields_perturbation_storage": fields_p,
            "tolerance_rho_E": 1e-5,
            "within_tolerance": bool(fields["rho"]["max_rel"] <= 1e-5 and fields["E"]["max_rel"] <= 1e-5
                                     and fields_p["rho"]["max_rel"] <= 1e-5
                                     and fields_p["E"]["max_rel"] <= 1e-5)}


def run_cpu_baseline():
    import numpy as np
    import torch

    import oracle
    import workloads as wl

    nthreads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        nthreads = min(nthreads, int(env))
    torch.set_num_threads(nthreads)
    grid, q, _ = wl.convection_3d(NX, NY, NZ)
    b = 128
    sub = grid.copy(nx=b, ny=b)
    qs = np.zeros(sub.shape)
    sub.interior(qs)[...] = grid.interior(q)[:, :, :b, :b]
    del q
    dt = oracle.cfl_dt(qs, sub, CFL)
    # steps of the same dt until about 15 s of host time (4 to 24 steps), so the
    # sample stays bounded on slow hosts
    nsteps, el = 0, 0.0
    t0 = time.perf_counter()
    while nsteps < 24 and (nsteps < 4 or el < 15.0):
        qs = oracle.run(qs, sub, dt, 1)
        qs = qs.numpy() if hasattr(qs, "numpy") else qs
        nsteps += 1
        el = time.perf_counter() - t0
    return {
        "value": b * b * NZ * nsteps / el, "unit": "cell-updates/s", "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": f"{nsteps} SSP-RK3 steps (FP64) of a {b}x{b}x{NZ} column block cut from the "
                  f"same initial state, periodic in x and y ({el:.1f} s)",
    }


def run_bubble2d(steps: int = 20, repeats: int = 5):
    """The 2-D dry bubble (64x64, FP64), 20 steps of the device-dt step: a
    parity-size case, cache- and launch-bound, reported in cell-updates/s."""
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    grid, q = wl.bubble_2d()
    dg = snap.device_grid(grid)
    q0 = torch.as_tensor(q).cuda()
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    qd = q0.clone()
    snap.snap_rk3_steps_cfl(dg, qd, CFL, 3, work)

    def call():
        qd.copy_(q0)
        snap.snap_rk3_steps_cfl(dg, qd, CFL, steps, work)

    times = _timed(call, repeats)
    snap.snap_rk3_steps_status(dg, work)
    el = _median(times)
    # the same call captured once in a HIP graph (it launches kernels only) and
    # replayed: one graph launch instead of the 60 stage launches and the
    # reduction's, which dominate at this size
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        qd.copy_(q0)
        snap.snap_rk3_steps_cfl(dg, qd, CFL, steps, work)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        snap.snap_rk3_steps_cfl(dg, qd, CFL, steps, work)

    def gcall():
        qd.copy_(q0)
        graph.replay()

    gtimes = _timed(gcall, repeats)
    snap.snap_rk3_steps_status(dg, work)
    gel = _median(gtimes)
    del graph
    cells = grid.nx * grid.nz
    return {"workload": "2-D dry bubble 64x64 (20 x 10 km), FP64, 20 SSP-RK3 steps, CFL 0.9",
            "value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el / steps * 1e3,
            "steps": steps, "repeats": repeats, "spread": _spread(times),
            "graph": {"value": cells * steps / gel, "ms_per_step": gel / steps * 1e3,
                      "spread": _spread(gtimes)}}


def _oracle_threads():
    import torch

    nthreads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        nthreads = min(nthreads, int(env))
    torch.set_num_threads(nthreads)
    return torch.get_num_threads()


def run_cpu_oracle_sections():
    """The FP64 oracle (PyTorch CPU) on bounded samples of the other workloads:
    all 20 steps of the 2-D bubble; 1 step of a 64 x 64 x 256 column slab of
    the Jovian column (4 passive tracers); one step of each of the 64 ensemble
    members in turn; and the backward / forward time of 2 steps of a 64 x 64 x
    128 sub-domain of the gradient workload (torch autograd through the oracle)."""
    import numpy as np
    import torch

    import oracle
    import workloads as wl

    cores = _oracle_threads()
    out = {"cores": cores, "kind": "oracle"}

    grid, q = wl.bubble_2d()
    dt = oracle.cfl_dt(q, grid, CFL)
    t0 = time.perf_counter()
    oracle.run(q, grid, dt, 20)
    el = time.perf_counter() - t0
    out["bubble2d"] = {"value": grid.nx * grid.nz * 20 / el, "unit": "cell-updates/s",
                       "sample": f"all 20 steps of the 64x64 bubble ({el:.2f} s)"}

    # a 64 x 64 column slab: at 128 x 128 the oracle's whole-array temporaries
    # (tens of GB) slowed it about threefold per cell on a 64 GB host
    grid, q = wl.jovian_3d(nx=64, ny=64, nz=256)
    dt = oracle.cfl_dt(q, grid, CFL)
    t0 = time.perf_counter()
    oracle.run(q, grid, dt, 1)
    el = time.perf_counter() - t0
    del q
    out["jovian_slab"] = {"value": 64 * 64 * 256 / el, "unit": "cell-updates/s",
                          "sample": f"1 step of a 64x64x256 slab of the Jovian column, 4 passive "
                                    f"tracers ({el:.1f} s)"}

    members = wl.ensemble_2d(64, seed=4)
    cells, el = 0, 0.0
    for g, qm in members:
        dtm = oracle.cfl_dt(qm, g, CFL)
        t0 = time.perf_counter()
        oracle.rk3_step(qm, g, dtm)
        el += time.perf_counter() - t0
        cells += g.nx * g.nz
    out["ensemble"] = {"value": cells / el, "unit": "cell-updates/s",
                       "sample": f"one step of each of the 64 members in turn ({el:.1f} s)"}

    grid, base, dth, vel, dp = wl.convection_flow_3d(64, 64, 128, lx=5e3, ly=5e3, lz=10e3)
    q = wl.state_from_theta(grid, base, torch.as_tensor(dth), torch.as_tensor(vel),
                            torch.as_tensor(dp)).numpy()
    dt = oracle.cfl_dt(q, grid, CFL)
    n = 2
    t0 = time.perf_counter()
    oracle.run(q, grid, dt, n)
    t_fwd = time.perf_counter() - t0
    qt = torch.as_tensor(q)
    g0 = 3
    qi = qt[:, g0:g0 + grid.nz, g0:g0 + grid.ny, g0:g0 + grid.nx].clone().requires_grad_(True)
    full = qt.clone()
    full[:, g0:g0 + grid.nz, g0:g0 + grid.ny, g0:g0 + grid.nx] = qi
    outq = oracle.run(full, grid, dt, n)
    top = outq[:, g0 + grid.nz - 16:g0 + grid.nz, g0:g0 + grid.ny, g0:g0 + grid.nx]
    L = 0.5 * ((top[1] ** 2 + top[2] ** 2 + top[3] ** 2) / top[0]).sum()
    t0 = time.perf_counter()
    L.backward()
    t_bwd = time.perf_counter() - t0
    out["adjoint_subdomain"] = {"forward_s": t_fwd, "backward_s": t_bwd,
                                "adjoint_forward_ratio": t_bwd / t_fwd,
                                "sample": "2 steps of a 64x64x128 sub-domain of the gradient workload "
                                          "(the backward: torch autograd through the oracle)"}
    return out


def run_profile_target(name: str):
    """A short run of one section's kernels, for rocprofv3 (counters or trace):
    'jovian' (3 device-dt steps of the passive and of the mixture Jovian
    column), 'kessler' (3 steps of the Kessler workload with falling rain),
    'satadj' (3 saturation adjustments), 'adjoint' (3 RK3 adjoint steps of the
    256x256x128 convection state, FP32 and FP64, stage states kept)."""
    import torch

    import paper_1901_02955_amd as snap
    import workloads as wl

    if name == "jovian":
        run_jovian(3, 1, repeats=1)
        run_jovian(3, 1, mixture=True, repeats=1)
    elif name == "kessler":
        run_jovian_kessler(3, 1, repeats=1)
    elif name == "satadj":
        run_jovian_satadj(3, 1, repeats=1)
    elif name == "adjoint":
        grid, q, _ = wl.convection_3d(NX, NY, NZ)
        for dtype in (torch.float32, torch.float64):
            dg = snap.device_grid(grid, dtype=dtype)
            qn = torch.as_tensor(q).to(dtype).cuda()
            dt = snap.snap_cfl_dt(dg, qn, CFL, snap.workspace(dg, snap.SNAP_OP_CFL))
            stages = snap.workspace(dg, snap.SNAP_OP_RK3)
            snap.snap_rk3_step(dg, qn.clone(), dt, stages)
            aw = snap.workspace(dg, snap.SNAP_OP_RK3_ADJ)
            qb = torch.as_tensor(wl.seeded_normal(grid.interior_shape, 3)).to(dtype).cuda()
            for _ in range(3):
                snap.snap_rk3_step_adjoint_stages(dg, qn, stages, dt, qb, aw)
            torch.cuda.synchronize()
            del qn, stages, aw, qb
            torch.cuda.empty_cache()
    else:
        raise SystemExit(f"unknown profile target {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the Jovian, ensemble and adjoint sections")
    ap.add_argument("--variant", choices=("both", "f64", "f32"), default="both",
                    help="f64 or f32 alone (for profiling runs); the JSON line then carries that form")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one device-to-device copy of 512 MiB (a known byte count "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--profile", choices=("jovian", "kessler", "satadj", "adjoint"),
                    help="run only a short invocation of that section's kernels (for rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU kernel here; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile:
        run_profile_target(args.profile)
        return
    if args.variant == "f32":
        f32 = run_gpu(torch.float32, args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": f32["value"], "unit": "cell-updates/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": f32["ms_per_step"], "dtype": "f32",
                          "roofline": f32["roofline"],
                          "stage_kernel_avg_ms": f32["stage_kernel_avg_ms"]}), flush=True)
        return
    t_start = time.perf_counter()

    def progress(section):
        print(f"[bench] {section} done at {time.perf_counter() - t_start:.1f} s", file=sys.stderr,
              flush=True)

    f64 = run_gpu(torch.float64, args.steps, args.warmup)
    progress("headline f64")
    out = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3-D dry convection 256x256x128 (20x20x10 km), FP64, 5 conserved vars, "
                        "periodic x/y, rigid lids, CFL 0.9 (dt per step, formed on the device), WENO5+LMARS, SSP-RK3",
            "nx": NX, "ny": NY, "nz": NZ, "nvar": 5, "cfl": CFL,
        },
        "repeats": f64["repeats"],
        "spread": f64["spread"],
        "roofline": f64["roofline"],
        "hbm_roofline": f64["hbm_roofline"],
        "hbm_target": {
            "target_frac": 0.6,
            "algorithmic_bytes_frac": f64["hbm_roofline"]["frac"],
            "measured_bytes_frac": f64["hbm_roofline"]["measured_frac"],
            "why_below": "the fused stage kernel moves only the algorithmic state passes (face "
                         "states, fluxes and the divergence stay on chip) and is bound by "
                         "vector-ALU issue, not by HBM: see valu_utilisation and roofline",
        },
        "valu_utilisation": f64["valu_utilisation"],
        "traffic_source": "rocprofv3 FETCH_SIZE / WRITE_SIZE of the stage kernel, scaled by a "
                          "512 MiB copy (profiles/stage_kernel_traffic.txt); null unless taken on "
                          "the current kernel sources",
        "stage_kernel_avg_ms": f64["stage_kernel_avg_ms"],
    }
    if not args.no_f32 and args.variant == "both":
        f32 = run_gpu(torch.float32, args.steps, args.warmup)
        out["variants"] = {"f32": {
            "value": f32["value"], "ms_per_step": f32["ms_per_step"], "dtype": "f32",
            "repeats": f32["repeats"], "spread": f32["spread"],
            "stage_kernel_avg_ms": f32["stage_kernel_avg_ms"], "roofline": f32["roofline"],
            "hbm_roofline": f32["hbm_roofline"], "valu_utilisation": f32["valu_utilisation"],
        }}
        out["f32_speedup"] = f32["value"] / f64["value"]
        progress("f32")
        f32p = run_gpu(torch.float32, args.steps, args.warmup, perturbation=True)
        out["variants"]["f32_perturbation"] = {
            "value": f32p["value"], "ms_per_step": f32p["ms_per_step"], "dtype": "f32",
            "storage": "rho - rhobar_k, E - pbar_k / (gamma - 1)",
            "repeats": f32p["repeats"], "spread": f32p["spread"],
            "stage_kernel_avg_ms": f32p["stage_kernel_avg_ms"], "roofline": f32p["roofline"],
            "hbm_roofline": f32p["hbm_roofline"],
        }
        progress("f32 perturbation storage")
        out["f32_error_vs_f64"] = run_fp32_error()
        progress("f32 error")
    if not args.only_headline:
        out["jovian"] = run_jovian(50, 3)
        out["jovian_mixture"] = run_jovian(50, 3, mixture=True)
        out["jovian_mixture"]["cost_vs_passive"] = (out["jovian"]["value"]
                                                    / out["jovian_mixture"]["value"])
        progress("jovian")
        out["jovian_kessler"] = run_jovian_kessler(20, 2)
        progress("jovian kessler")
        out["jovian_satadj"] = run_jovian_satadj(20, 2)
        progress("jovian saturation adjustment")
        out["hllc"] = {}
        for name, dt_, ref in (("f64", torch.float64, f64), ("f32", torch.float32, out.get("variants", {}).get("f32"))):
            h = run_gpu(dt_, 30, 3, hllc=True)
            out["hllc"][name] = {"value": h["value"], "ms_per_step": h["ms_per_step"],
                                 "repeats": h["repeats"], "spread": h["spread"],
                                 "stage_kernel_avg_ms": h["stage_kernel_avg_ms"],
                                 "roofline": h["roofline"],
                                 "cost_vs_lmars": (ref["value"] / h["value"]) if ref else None}
        progress("hllc")
        out["ensemble"] = run_ensemble(20)
        progress("ensemble")
        out["bubble2d"] = run_bubble2d()
        out["adjoint"] = run_adjoint()
        progress("adjoint")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline()
        progress("cpu baseline")
        if not args.only_headline:
            out["cpu_oracle_sections"] = run_cpu_oracle_sections()
            progress("cpu oracle sections")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
