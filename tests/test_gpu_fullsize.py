"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (the same grids, element types, tile shapes and z-chunks):

* right-hand side of the 3-D convection grid 256 x 256 x 128 (FP64 and FP32)
  and of the Jovian column 512 x 512 x 256 with four tracers (FP32, passive
  and mixture equation of state), compared with the FP64 oracle on sampled
  8 x 8 x 8 blocks. The oracle evaluates each block from the ghost-filled full
  state (its own fill), so every sample sees exactly the inputs the kernel
  saw. The blocks sit on the periodic seams and both walls, straddle tile
  edges (multiples of 16 cells) and z-chunk edges, and at seeded positions;
* one full-size SSP-RK3 step, through properties that hold at any size:
  mass and horizontal momentum are conserved (periodic in x and y, rigid
  lids), and the step equals three right-hand sides combined on the host;
* the right-hand-side adjoint of the full grid for a cotangent that is
  nonzero on a 4 x 4 x 4 block only: equal to the oracle's reverse mode on
  the surrounding 20 x 20 x 20 block, and exactly zero outside it;
* the Jovian column with six tracers and falling rain: the right-hand side
  with the sedimentation terms (blocks away from the walls), and the Kessler
  step on the benchmark's own state (sampled blocks);
* the adjoints of the Kessler step and of the saturation adjustment on the
  benchmarks' own states with a full-size cotangent (sampled blocks: both are
  pointwise, so a block's cotangent depends on the block alone);
* the benchmark's ensemble of 64 bubbles: every tile variant batched against
  separate steps, and the 2-D right-hand side at each member size against the
  oracle cell by cell.

States are seeded smooth-plus-noise perturbations of the hydrostatic base
state, so that every term of every field is active.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_02955_amd as snap
import workloads as wl
from tests.test_gpu_fp32 import RHS32_TOL
from tests.test_gpu_parity import TOL64

pytestmark = pytest.mark.gpu

G = 3      # ghost layers
B = 8      # sampled block edge


def sample_blocks(grid):
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    h = B // 2
    out = [(0, 0, 0),                                  # x/y seams, ground
           (nx - B, ny - B, nz - B),                   # x/y seams, lid
           (nx - B, 0, nz // 2 - h),                   # half height (chunk edge)
           (16 - h, 32 - h, nz // 4 - h),              # tile corner, quarter height
           (nx // 2 - h, ny - B, 3 * nz // 4 - h),     # three-quarter height
           (48 - h, ny // 2 - h, 0)]                   # tile edge at the ground
    rng = np.random.default_rng(11)
    for _ in range(2):
        out.append((int(rng.integers(0, nx - B + 1)), int(rng.integers(0, ny - B + 1)),
                    int(rng.integers(0, nz - B + 1))))
    return out


def sub_grid(grid, k0, n):
    """Grid of an n x n x n block whose lowest level is k0 (references sliced)."""
    return grid.copy(nx=n, ny=n, nz=n,
                     rhobar_cell=np.asarray(grid.rhobar_cell)[k0:k0 + n + 2 * G],
                     pbar_cell=np.asarray(grid.pbar_cell)[k0:k0 + n + 2 * G],
                     rhobar_face=np.asarray(grid.rhobar_face)[k0:k0 + n + 1],
                     pbar_face=np.asarray(grid.pbar_face)[k0:k0 + n + 1])


def padded_block(qf, i0, j0, k0, n):
    return qf[:, k0:k0 + n + 2 * G, j0:j0 + n + 2 * G, i0:i0 + n + 2 * G].contiguous()


def check_rhs_blocks(grid, q, dtype, tol, label, blocks=None, z_open=False):
    """GPU right-hand side of the full grid against the oracle on sampled blocks
    (z_open: the blocks' z ends are not walls, for terms that close the walls)."""
    print(f"[fullsize] {label}: {grid.nx}x{grid.ny}x{grid.nz} nvar {grid.nvar} {dtype}",
          flush=True)
    qt = torch.as_tensor(q).to(dtype)
    dg = snap.device_grid(grid, dtype=dtype)
    qd = qt.cuda()
    rhs = torch.empty(dg.interior_shape, dtype=dtype, device="cuda")
    snap.snap_rhs(dg, qd, rhs)
    torch.cuda.synchronize()
    del qd
    qf = oracle.fill_ghosts(qt.double(), grid)      # the oracle's own ghost fill
    del qt
    got, ref = [], []
    for (i0, j0, k0) in (blocks or sample_blocks(grid)):
        sg = sub_grid(grid, k0, B)
        if z_open:
            sg = sg.copy(bc=(grid.bc[0], grid.bc[1], wl.BC_PERIODIC))
        r = oracle.rhs_filled(padded_block(qf, i0, j0, k0, B), sg).numpy()
        g = rhs[:, k0:k0 + B, j0:j0 + B, i0:i0 + B].double().cpu().numpy()
        ref.append(r.reshape(grid.nvar, -1))
        got.append(g.reshape(grid.nvar, -1))
    del rhs, qf
    torch.cuda.empty_cache()
    ref = np.concatenate(ref, axis=1)
    got = np.concatenate(got, axis=1)
    bad = []
    for m in range(grid.nvar):
        scale = float(np.max(np.abs(ref[m])))
        err = float(np.max(np.abs(got[m] - ref[m])))
        print(f"   field {m}: max|ref| {scale:.3e}  error / max|ref| {err / scale:.2e}", flush=True)
        assert scale > 0.0
        if not err <= tol * scale:
            bad.append(m)
    assert not bad, (label, bad)


@pytest.fixture(scope="module")
def convection():
    grid, _ = wl.dry_grid(256, 256, 128, 20e3, 20e3, 10e3)
    return grid, wl.random_smooth_state(grid, seed=31)


@pytest.fixture(scope="module")
def jovian():
    grid, _ = wl.jovian_3d(nx=512, ny=512, nz=256)
    q = wl.random_smooth_state(grid, seed=32, amp_q=2e-3)
    return grid, q


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rhs_fullsize_convection(convection, dtype):
    grid, q = convection
    tol = TOL64 if dtype == torch.float64 else RHS32_TOL
    check_rhs_blocks(grid, q, dtype, tol, "convection rhs")


@pytest.mark.parametrize("mixture", [False, True], ids=["passive", "mixture"])
def test_rhs_fullsize_jovian_fp32(jovian, mixture):
    grid, q = jovian
    if mixture:
        grid = wl.with_mixture(grid, wl.condensable_species(wl.jovian_base().cp - wl.jovian_base().rd,
                                                            wl.JOVIAN_MU))
    check_rhs_blocks(grid, q, torch.float32, RHS32_TOL, "jovian rhs " + ("mixture" if mixture
                                                                       else "passive"))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rk3_fullsize_conserves_and_composes(convection, dtype):
    grid, q = convection
    print(f"[fullsize] rk3 {grid.nx}x{grid.ny}x{grid.nz} {dtype}", flush=True)
    dg = snap.device_grid(grid, dtype=dtype)
    y0 = torch.as_tensor(q).to(dtype).cuda()
    sums_work = snap.workspace(dg, snap.SNAP_OP_SUMS)
    dt = snap.snap_cfl_dt(dg, y0.clone(), 0.9, snap.workspace(dg, snap.SNAP_OP_CFL))

    def interior(t):
        return t[:, G:G + grid.nz, G:G + grid.ny, G:G + grid.nx]

    # three right-hand sides combined on the host (torch arithmetic)
    R = torch.empty(dg.interior_shape, dtype=dtype, device="cuda")
    ya = y0.clone()
    snap.snap_rhs(dg, ya, R)
    y1 = y0.clone()
    interior(y1).copy_(interior(y0) + dt * R)
    snap.snap_rhs(dg, y1, R)
    y2 = y0.clone()
    interior(y2).copy_(0.75 * interior(y0) + 0.25 * (interior(y1) + dt * R))
    snap.snap_rhs(dg, y2, R)
    host = (1.0 / 3.0) * interior(y0) + (2.0 / 3.0) * (interior(y2) + dt * R)
    del ya, y1, y2, R
    # the library's step, as the benchmark calls it
    qs = y0.clone()
    s0 = snap.snap_conservation_sums(dg, qs, sums_work)
    snap.snap_rk3_step(dg, qs, dt, snap.workspace(dg, snap.SNAP_OP_RK3))
    s1 = snap.snap_conservation_sums(dg, qs, sums_work)
    step = interior(qs)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for m in range(grid.nvar):
        scale = float(interior(y0)[m].abs().max())
        diff = float((step[m] - host[m]).abs().max())
        moved = float((step[m] - interior(y0)[m]).abs().max())
        print(f"   field {m}: step vs host {diff / scale:.2e}, change {moved / scale:.2e}",
              flush=True)
        assert diff <= tol * scale, (m, diff / scale)
        assert moved > 100 * diff, (m, moved / scale)   # the step moved far more than that
    # mass and horizontal momentum: fluxes telescope, the lids carry no mass
    # and no horizontal force acts
    qi = np.abs(wl.Grid.interior(grid, np.asarray(q))).reshape(grid.nvar, -1).sum(axis=1)
    ctol = 1e-12 if dtype == torch.float64 else 1e-6
    for m in (0, 1, 2):
        print(f"   sum of field {m}: {s0[m]:.15e} -> {s1[m]:.15e}", flush=True)
        assert abs(s1[m] - s0[m]) <= ctol * qi[m], (m, s0[m], s1[m])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rhs_adjoint_fullsize_local(convection, dtype):
    """Cotangent on a 4^3 block: q_bar equals the oracle's reverse mode on the
    surrounding 20^3 block (whose ghosts are held fixed: none of them is
    reached), and is exactly zero everywhere else."""
    grid, q = convection
    print(f"[fullsize] adjoint {grid.nx}x{grid.ny}x{grid.nz} {dtype}", flush=True)
    n, s = 20, 4
    dg = snap.device_grid(grid, dtype=dtype)
    qt = torch.as_tensor(q).to(dtype)
    qf = oracle.fill_ghosts(qt.double(), grid)
    work = snap.workspace(dg, snap.SNAP_OP_RHS_ADJ)
    tol = 1e-11 if dtype == torch.float64 else 1e-3
    for (i0, j0, k0) in [(100, 60, 40), (250 - n, 3, 90)]:
        print(f"   block at ({i0}, {j0}, {k0})", flush=True)
        a = (n - s) // 2
        rbar = torch.zeros(dg.interior_shape, dtype=torch.float64)
        local = torch.as_tensor(wl.seeded_normal((grid.nvar, s, s, s), 7 + i0))
        rbar[:, k0 + a:k0 + a + s, j0 + a:j0 + a + s, i0 + a:i0 + a + s] = local
        qb = torch.empty(dg.interior_shape, dtype=dtype, device="cuda")
        snap.snap_rhs_adjoint(dg, qt.cuda(), rbar.to(dtype).cuda(), qb, work)
        qb = qb.double().cpu()
        # oracle: reverse mode of the block's right-hand side w.r.t. its interior
        sub = padded_block(qf, i0, j0, k0, n)
        sg = sub_grid(grid, k0, n)
        qi = sub[:, G:G + n, G:G + n, G:G + n].clone().requires_grad_(True)
        full = sub.clone()
        full[:, G:G + n, G:G + n, G:G + n] = qi
        r = oracle.rhs_filled(full, sg)
        rb_sub = rbar[:, k0:k0 + n, j0:j0 + n, i0:i0 + n].to(dtype).double()
        (ref,) = torch.autograd.grad(r, qi, rb_sub)
        got = qb[:, k0:k0 + n, j0:j0 + n, i0:i0 + n]
        for m in range(grid.nvar):
            scale = float(ref[m].abs().max())
            err = float((got[m] - ref[m]).abs().max())
            print(f"      field {m}: error / max|ref| {err / scale:.2e}", flush=True)
            assert err <= tol * scale, (m, err / scale)
        outside = qb.clone()
        outside[:, k0:k0 + n, j0:j0 + n, i0:i0 + n] = 0.0
        assert float(outside.abs().max()) == 0.0


@pytest.fixture(scope="module")
def jovian_kessler():
    return wl.jovian_kessler_3d(sediment=True)


def interior_blocks(grid):
    """Sampled blocks whose z ends are not walls."""
    return [(b[0], b[1], min(max(b[2], 1), grid.nz - B - 1)) for b in sample_blocks(grid)]


def test_rhs_fullsize_jovian_sedimentation_fp32(jovian_kessler):
    """Six tracers under the mixture equation of state with the water and
    ammonia rain falling (the benchmark's microphysics workload): the
    right-hand side with the sedimentation terms on blocks away from the
    walls (the walls' closure is covered at small sizes)."""
    grid, _, _ = jovian_kessler
    q = wl.random_smooth_state(grid, seed=33, amp_q=2e-3)
    check_rhs_blocks(grid, q, torch.float32, RHS32_TOL, "jovian rhs with sedimentation",
                     blocks=interior_blocks(grid), z_open=True)


def test_kessler_fullsize_fp32(jovian_kessler):
    """The Kessler step on the benchmark's own state (vapour supersaturated
    aloft, cloud and rain seeded) against the oracle on sampled blocks; the
    other fields are left bit for bit."""
    grid, q, kes = jovian_kessler
    dt = 0.5
    print(f"[fullsize] kessler {grid.nx}x{grid.ny}x{grid.nz} nvar {grid.nvar} fp32", flush=True)
    qt = torch.as_tensor(q).float()
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = qt.cuda()
    snap.snap_kessler_step(dg, qd, dt, kes)
    got_full = qd
    got, ref, orig = [], [], []
    for (i0, j0, k0) in sample_blocks(grid):
        blk = padded_block(qt.double(), i0, j0, k0, B)
        r = oracle.kessler_step(blk, sub_grid(grid, k0, B), dt, kes)
        ref.append(r[:, G:G + B, G:G + B, G:G + B].reshape(grid.nvar, -1).numpy())
        sl = (slice(None), slice(k0 + G, k0 + G + B), slice(j0 + G, j0 + G + B),
              slice(i0 + G, i0 + G + B))
        got.append(got_full[sl].double().cpu().reshape(grid.nvar, -1).numpy())
        orig.append(qt[sl].double().reshape(grid.nvar, -1).numpy())
    del qd, got_full
    torch.cuda.empty_cache()
    ref, got, orig = (np.concatenate(x, axis=1) for x in (ref, got, orig))
    assert np.array_equal(got[:5], orig[:5])
    for m in range(5, grid.nvar):
        scale = float(np.max(np.abs(ref[m])))
        err = float(np.max(np.abs(got[m] - ref[m])))
        moved = float(np.max(np.abs(ref[m] - orig[m])))
        print(f"   tracer {m - 5}: error / max|ref| {err / scale:.2e}, change {moved / scale:.1e}",
              flush=True)
        assert err <= 1e-6 * scale, (m, err / scale)


def pattern_cotangent(shape, device="cpu", origin=(0, 0, 0)):
    """A seeded cotangent of small exact values, ((7 i + 13 j + 29 k + 31 m) mod
    17 - 8) / 8 at variable m and interior cell (i, j, k) (offset by origin),
    identical in FP32 on the device and in FP64 on the host, so a sampled
    block of the full-size array can be rebuilt without storing it."""
    nv, nz, ny, nx = shape
    i0, j0, k0 = origin
    m = torch.arange(nv, device=device).view(nv, 1, 1, 1)
    k = torch.arange(k0, k0 + nz, device=device).view(1, nz, 1, 1)
    j = torch.arange(j0, j0 + ny, device=device).view(1, 1, ny, 1)
    i = torch.arange(i0, i0 + nx, device=device).view(1, 1, 1, nx)
    return (((7 * i + 13 * j + 29 * k + 31 * m) % 17) - 8).to(torch.float32) / 8.0


def check_pointwise_adjoint(grid, q, run_gpu, run_oracle, tag):
    """A pointwise operation's adjoint on the full FP32 state with the pattern
    cotangent, against the oracle's on sampled blocks (every cell's cotangent
    depends on that cell alone): within 1e-5 of each field's largest magnitude."""
    qt = torch.as_tensor(q).float()
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = qt.cuda()
    qb = pattern_cotangent(dg.interior_shape, device="cuda").contiguous()
    print(f"[fullsize] {tag} adjoint {grid.nx}x{grid.ny}x{grid.nz} nvar {grid.nvar} fp32", flush=True)
    run_gpu(dg, qd, qb)
    got, ref = [], []
    for (i0, j0, k0) in sample_blocks(grid):
        blk = padded_block(qt.double(), i0, j0, k0, B)
        qbb = pattern_cotangent((grid.nvar, B, B, B), origin=(i0, j0, k0)).double().numpy()
        ref.append(run_oracle(blk, sub_grid(grid, k0, B), qbb).reshape(grid.nvar, -1).numpy())
        got.append(qb[:, k0:k0 + B, j0:j0 + B, i0:i0 + B].double().cpu().reshape(grid.nvar, -1)
                   .numpy())
    del qd, qb
    torch.cuda.empty_cache()
    ref, got = np.concatenate(ref, axis=1), np.concatenate(got, axis=1)
    for m in range(grid.nvar):
        scale = float(np.max(np.abs(ref[m])))
        err = float(np.max(np.abs(got[m] - ref[m])))
        print(f"   field {m}: error / max|ref| {err / scale:.2e}", flush=True)
        assert err <= 1e-5 * scale, (m, err / scale)


def test_kessler_adjoint_fullsize_fp32(jovian_kessler):
    """The Kessler step's adjoint on the benchmark's own state and a full-size
    cotangent, against the oracle's autograd on sampled blocks."""
    grid, q, kes = jovian_kessler
    dt = 0.5

    def run_oracle(blk, sg, qbb):
        x = oracle.snap_oracle._interior(blk, sg).clone().requires_grad_(True)
        out = oracle.kessler_step(oracle.snap_oracle._with_interior(blk, sg, x), sg, dt, kes)
        (g,) = torch.autograd.grad(oracle.snap_oracle._interior(out, sg), x, torch.as_tensor(qbb))
        return g

    check_pointwise_adjoint(grid, q, lambda dg, qd, qb: snap.snap_kessler_step_adjoint(dg, qd, dt, kes, qb),
                            run_oracle, "kessler")


def test_saturation_adjust_adjoint_fullsize_fp32():
    """The saturation adjustment's adjoint on the benchmark's own state and a
    full-size cotangent, against the oracle's implicit-function derivative on
    sampled blocks."""
    grid, q, adj = wl.jovian_satadj_3d()
    check_pointwise_adjoint(
        grid, q, lambda dg, qd, qb: snap.snap_saturation_adjust_adjoint(dg, qd, adj, qb),
        lambda blk, sg, qbb: oracle.saturation_adjust_adjoint(blk, sg, adj, qbb), "saturation adjustment")


def test_ensemble_fullsize_batched_equals_separate():
    """The benchmark's 64 uneven bubbles (FP32): every tile variant the tuner
    chooses from, batched, against separate steps (bit for bit for the
    default tile shape, within a few ulp for the others)."""
    from paper_1901_02955_amd import tuner
    members = wl.ensemble_2d(64, seed=4)
    grids = [snap.device_grid(g, dtype=torch.float32) for g, _ in members]
    print(f"[fullsize] ensemble of {len(grids)}: {sum(g.nx * g.nz for g in grids)} cells",
          flush=True)
    cw = snap.workspace(grids[0], snap.SNAP_OP_CFL)
    q0 = [torch.as_tensor(q).float().cuda() for _, q in members]
    dts = [snap.snap_cfl_dt(g, q.clone(), 0.9, cw) for g, q in zip(grids, q0)]
    ref = []
    for dg, q, dt in zip(grids, q0, dts):
        qd = q.clone()
        snap.snap_rk3_step(dg, qd, dt, snap.workspace(dg, snap.SNAP_OP_RK3))
        ref.append(qd)
    work = snap.batched_workspace(grids)
    for v, shape in tuner.candidates(grids):
        print(f"   variant {v} {shape}", flush=True)
        qs = [q.clone() for q in q0]
        snap.snap_rk3_step_batched(grids, qs, dts, work, v, 0)
        for m, (g, _) in enumerate(members):
            a = g.interior(qs[m].cpu().double().numpy())
            b = g.interior(ref[m].cpu().double().numpy())
            if v == 0:
                assert np.array_equal(a, b), (v, m)
            else:
                for k in range(g.nvar):
                    scale = max(float(np.abs(b[k]).max()), 1e-300)
                    assert float(np.abs(a[k] - b[k]).max()) <= 1e-6 * scale, (v, m, k)


@pytest.mark.parametrize("size", wl.ENSEMBLE_SIZES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rhs_fullsize_bubble_member(size, dtype):
    """The 2-D right-hand side at each member size of the ensemble, every cell
    against the oracle."""
    nx, nz = size
    g, _ = wl.bubble_2d(nx=nx, nz=nz)
    q = wl.random_smooth_state(g, seed=40 + nx)
    print(f"[fullsize] bubble member {nx}x{nz} {dtype}", flush=True)
    qt = torch.as_tensor(q).to(dtype)
    dg = snap.device_grid(g, dtype=dtype)
    rhs = torch.empty(dg.interior_shape, dtype=dtype, device="cuda")
    snap.snap_rhs(dg, qt.cuda(), rhs)
    ref = oracle.rhs(qt.double().numpy(), g).numpy()
    got = rhs.double().cpu().numpy()
    tol = TOL64 if dtype == torch.float64 else RHS32_TOL
    for m in range(g.nvar):
        scale = float(np.max(np.abs(ref[m])))
        err = float(np.max(np.abs(got[m] - ref[m])))
        if scale == 0.0:          # y momentum of an x-z problem
            print(f"   field {m}: identically zero, error {err:.2e}", flush=True)
            assert err == 0.0
            continue
        print(f"   field {m}: error / max|ref| {err / scale:.2e}", flush=True)
        assert err <= tol * scale, (m, err / scale)


def test_saturation_adjust_fullsize_fp32():
    """The saturation adjustment on the benchmark's own 512 x 512 x 256 state
    (water and ammonia vapour supersaturated aloft, clouds seeded) against the
    oracle on sampled blocks; the other fields are left bit for bit."""
    grid, q, adj = wl.jovian_satadj_3d()
    print(f"[fullsize] saturation adjustment {grid.nx}x{grid.ny}x{grid.nz} nvar {grid.nvar} fp32",
          flush=True)
    qt = torch.as_tensor(q).float()
    dg = snap.device_grid(grid, dtype=torch.float32)
    qd = qt.cuda()
    snap.snap_saturation_adjust(dg, qd, adj)
    got, ref, orig = [], [], []
    for (i0, j0, k0) in sample_blocks(grid):
        blk = padded_block(qt.double(), i0, j0, k0, B)
        r = oracle.saturation_adjust(blk, sub_grid(grid, k0, B), adj)
        ref.append(r[:, G:G + B, G:G + B, G:G + B].reshape(grid.nvar, -1).numpy())
        sl = (slice(None), slice(k0 + G, k0 + G + B), slice(j0 + G, j0 + G + B),
              slice(i0 + G, i0 + G + B))
        got.append(qd[sl].double().cpu().reshape(grid.nvar, -1).numpy())
        orig.append(qt[sl].double().reshape(grid.nvar, -1).numpy())
    del qd
    torch.cuda.empty_cache()
    ref, got, orig = (np.concatenate(x, axis=1) for x in (ref, got, orig))
    assert np.array_equal(got[:5], orig[:5])
    for m in range(5, grid.nvar):
        scale = float(np.max(np.abs(ref[m])))
        err = float(np.max(np.abs(got[m] - ref[m])))
        moved = float(np.max(np.abs(ref[m] - orig[m])))
        print(f"   tracer {m - 5}: error / max|ref| {err / scale:.2e}, change {moved / scale:.1e}",
              flush=True)
        assert err <= 1e-6 * scale, (m, err / scale)

