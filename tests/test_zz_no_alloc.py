"""snap_conservation_sums_noalloc (the library's own scratch, no workspace)
against snap_conservation_sums (the caller's workspace), through the C-ABI.

Both run the same kernels in the same fixed order, so the sums must agree bit
for bit. Two calls in a row on one GPU, the second on a smaller grid with fewer
variables, so that the second call runs over the partials the first one left
in the shared scratch; both element types.
"""
import numpy as np
import pytest
import torch

import paper_1901_02955_amd as snap
import workloads as wl

pytestmark = pytest.mark.gpu


def grids():
    big, _ = wl.dry_grid(37, 23, 19, 7400.0, 4600.0, 2850.0)
    big.ntracer = 4
    small, _ = wl.dry_grid(20, 1, 12, 4000.0, 1.0, 1800.0, bc=(0, 0, 1))
    small.dy = 1.0
    return [(big, wl.random_smooth_state(big, 51)), (small, wl.random_smooth_state(small, 52))]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_sums_equal_workspace_sums(dtype):
    for n, (grid, q) in enumerate(grids()):
        print(f"[no-alloc] call {n}: {grid.nx}x{grid.ny}x{grid.nz}, nvar {grid.nvar}, {dtype}",
              flush=True)
        dg = snap.device_grid(grid, dtype=dtype)
        qd = torch.as_tensor(q).to(dtype).cuda()
        got = snap.snap_conservation_sums_noalloc(dg, qd)
        ref = snap.snap_conservation_sums(dg, qd, snap.workspace(dg, snap.SNAP_OP_SUMS))
        assert got.shape == (grid.nvar,)
        assert np.array_equal(got, ref), (got, ref)
        # the sums are those of the interior (a property of the data, not of either path)
        vals = grid.interior(qd.double().cpu().numpy()).reshape(grid.nvar, -1)
        exact = vals.sum(axis=1)
        assert np.all(np.abs(got - exact) <= 1e-13 * np.abs(vals).sum(axis=1))
