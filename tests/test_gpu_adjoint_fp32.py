"""Single-precision right-hand-side adjoint: the y and z directions march
along their lines (one thread per line segment, a register window, no LDS)
where the variables fit, and otherwise use the tiled kernel of the x
direction.

* FP32 snap_rhs_adjoint against the oracle's FP64 J^T r_bar at the same
  (FP32-rounded) state and cotangent: within 1e-4 per field of the field's
  largest magnitude (single-precision evaluation of the face states and of
  the reverse sweep);
* the march against the tiled kernel (SNAP_ADJ_MARCH=0), both FP32, on the
  same inputs: within 1e-5 (the two sum the same contributions in different
  orders and share every other kernel), and on lines cut into several
  segments (SNAP_ADJ_MARCH_SEG) the same as on whole lines within that bar;
* both are reproducible bit for bit.
States at rest are left out, as in the FP64 adjoint tests.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
import workloads as wl
from tests import cases as C
from tests.test_gpu_parity import field_errors

pytestmark = pytest.mark.gpu

NAMES = ["2d_smooth_37x29_nt3", "2d_reflect_21x19", "2d_thin_19x2", "3d_smooth_35x21x19",
         "3d_tracers_20x18x24_nt4", "3d_linear_17x9x11", "3d_nt8_10x12x9",
         "3d_periodic_z_12x10x14", "3d_small_2x3x4", "3d_xwall_19x17x12",
         "3d_periodic_all_13x11x10"]


def long_case():
    """Lines long enough for several segments: 45 cells in y (walls), 70 in z."""
    g, _ = wl.dry_grid(16, 45, 70, 3200.0, 9000.0, 10500.0, bc=(0, 1, 1))
    g.ntracer = 1
    return C.Case("3d_long_16x45x70_nt1", g, wl.random_smooth_state(g, 51), 0.1)


def narrow_y_case():
    """Five cells in y (every row within 3 of a y edge: the z march folds no
    cell) and 14 levels."""
    g, _ = wl.dry_grid(12, 5, 14, 2400.0, 1000.0, 2800.0, bc=(1, 0, 1))
    return C.Case("3d_narrow_y_12x5x14", g, wl.random_smooth_state(g, 52), 0.1)


def narrow_x_cases():
    """Four cells in x (each cell has two copies in x: periodic, or mirrored
    at both walls), the rows and levels deep enough for the z march's fold."""
    out = []
    for bcx, seed in ((0, 53), (1, 54)):
        g, _ = wl.dry_grid(4, 9, 12, 800.0, 1800.0, 2400.0, bc=(bcx, 0, 1))
        out.append(C.Case(f"3d_narrow_x_4x9x12_bc{bcx}", g, wl.random_smooth_state(g, seed), 0.1))
    return out


def cases():
    for n in NAMES:
        yield C.build_case(n, dict(C.SPECS)[n])
    yield long_case()
    yield narrow_y_case()
    yield from narrow_x_cases()


class _env:
    """Set the library's adjoint switches for the calls inside the block."""

    def __init__(self, **kw):
        self.env = {k: str(v) for k, v in kw.items() if v is not None}

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.env}
        os.environ.update(self.env)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def adjoint32(c, rbar, march=True, seg=None, fold=True):
    with _env(SNAP_ADJ_MARCH=int(march), SNAP_ADJ_MARCH_SEG=seg, SNAP_ADJ_MARCH_FOLD=int(fold)):
        dg = snap.device_grid(c.grid, dtype=torch.float32)
        qd = torch.as_tensor(c.q).float().cuda()
        rb = torch.as_tensor(rbar).float().cuda()
        qb = torch.empty_like(rb)
        snap.snap_rhs_adjoint(dg, qd, rb, qb, snap.workspace(dg, snap.SNAP_OP_RHS_ADJ))
        return qb.cpu().double().numpy()


@pytest.mark.parametrize("c", list(cases()), ids=lambda c: c.name)
def test_rhs_adjoint_fp32(c):
    print(f"[adjoint32] {c.name}", flush=True)
    q32 = c.q.astype(np.float32).astype(np.float64)
    rbar = wl.seeded_normal(c.grid.interior_shape, 120).astype(np.float32).astype(np.float64)
    cr = C.Case(c.name, c.grid, q32, c.dt)
    march = adjoint32(cr, rbar)
    ref = oracle.rhs_adjoint(q32, c.grid, rbar).numpy()
    errs = field_errors(march, ref)
    print("   march vs oracle", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-4 for e in errs), errs
    tiled = adjoint32(cr, rbar, march=False)
    errs = field_errors(march, tiled)
    print("   march vs tiled", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-5 for e in errs), errs
    assert np.array_equal(march, adjoint32(cr, rbar))
    for seg in (7, 13):
        errs = field_errors(adjoint32(cr, rbar, seg=seg), march)
        assert all(e <= 1e-5 for e in errs), (seg, errs)
    # the z march's own fold of the cells away from the y and z edges against
    # the separate fold pass for every cell
    errs = field_errors(march, adjoint32(cr, rbar, fold=False))
    print("   march fold vs fold pass", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-5 for e in errs), errs


def rk3_adjoint32(c, qbar, march=True, fold=True):
    with _env(SNAP_ADJ_MARCH=int(march), SNAP_ADJ_MARCH_FOLD=int(fold)):
        dg = snap.device_grid(c.grid, dtype=torch.float32)
        qb = torch.as_tensor(qbar).float().cuda()
        snap.snap_rk3_step_adjoint(dg, torch.as_tensor(c.q).float().cuda(), c.dt, qb,
                                   snap.workspace(dg, snap.SNAP_OP_RK3_ADJ))
        return qb.cpu().double().numpy()


# The RK3 step adjoint folds its stages with the combinations of modes 3 and 4
# (out = alpha r_bar + beta J^T r_bar; out = alpha out + gam y + r_bar +
# beta J^T r_bar), which the z march then applies itself. Against the oracle
# the bar is that of the single-precision adjoint in test_gpu_adjoint.py
# (1e-3): the stage states are evaluated in single precision as well, and the
# reverse linearises the WENO5 weights at them. The three single-precision
# forms (the z march's fold, the separate fold pass, the tiled kernels) agree
# within 1e-5.
@pytest.mark.parametrize("c", [C.build_case(n, dict(C.SPECS)[n]) for n in
                               ("2d_smooth_37x29_nt3", "3d_smooth_35x21x19", "3d_xwall_19x17x12",
                                "3d_periodic_z_12x10x14", "3d_periodic_all_13x11x10")]
                         + [long_case(), narrow_y_case()] + narrow_x_cases(), ids=lambda c: c.name)
def test_rk3_step_adjoint_fp32_fold(c):
    print(f"[adjoint32] rk3 step {c.name}", flush=True)
    q32 = c.q.astype(np.float32).astype(np.float64)
    qbar = wl.seeded_normal(c.grid.interior_shape, 121).astype(np.float32).astype(np.float64)
    cr = C.Case(c.name, c.grid, q32, c.dt)
    folded = rk3_adjoint32(cr, qbar)
    ref = oracle.rk3_step_adjoint(q32, c.grid, c.dt, qbar).numpy()
    errs = field_errors(folded, ref)
    print("   vs oracle", ["%.2e" % e for e in errs], flush=True)
    assert all(e <= 1e-3 for e in errs), errs
    for kw in (dict(fold=False), dict(march=False)):
        other = rk3_adjoint32(cr, qbar, **kw)
        print("  ", kw, "vs oracle", ["%.2e" % e for e in field_errors(other, ref)], flush=True)
        errs = field_errors(folded, other)
        print("  ", kw, "vs folded", ["%.2e" % e for e in errs], flush=True)
        assert all(e <= 1e-5 for e in errs), (kw, errs)
