"""The 3-D stage launch sizes each chunk of levels by the dispatch pass that
runs it, when every compute unit holds one workgroup of each pass (256 column
tiles of 16 x 16 on a 256-compute-unit device): the first-dispatched
workgroup of a compute unit runs faster and gets more levels. Each level's
output depends only on the stage input, so every split must give the same
bits. Two SSP-RK3 steps of the 256 x 256 x 128 convection case are compared
under the default split, an even split, skewed splits and the split switched
off, in both element types.
"""
import os

import pytest
import torch

import paper_1901_02955_amd as snap
import workloads as wl

pytestmark = pytest.mark.gpu

ENV = "SNAP_STAGE_PASS_WEIGHTS"
SPLITS = {
    torch.float64: [None, "1,1", "2,1", "1,1.7", "off"],
    torch.float32: [None, "1,1,1", "1.6,1.2,1", "1,1,2", "off"],
}


@pytest.fixture
def restore_env():
    old = os.environ.get(ENV)
    yield
    if old is None:
        os.environ.pop(ENV, None)
    else:
        os.environ[ENV] = old


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_every_pass_split_gives_the_same_bits(dtype, restore_env):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    print(f"[pass-split] {dtype} 256x256x128, {cus} compute units", flush=True)
    grid, q, _ = wl.convection_3d(256, 256, 128)
    dg = snap.device_grid(grid, dtype=dtype)
    q0 = torch.as_tensor(q).to(dtype).cuda()
    work = snap.workspace(dg, snap.SNAP_OP_RK3)
    ref = None
    for w in SPLITS[dtype]:
        if w is None:
            os.environ.pop(ENV, None)
        else:
            os.environ[ENV] = w
        qd = q0.clone()
        for _ in range(2):
            snap.snap_rk3_step(dg, qd, 0.05, work)
        torch.cuda.synchronize()
        if ref is None:
            ref = qd
        else:
            assert torch.equal(ref, qd), f"split {w!r} changed the result"
    assert torch.isfinite(ref).all()
