"""The device-dt multi-step call (snap_rk3_steps_cfl) captured in a HIP graph
(torch.cuda.CUDAGraph on the current stream) and replayed: every replay equals
an eager call from the same state bit for bit, with eager calls on the same
workspace between the replays and a new state copied into the captured
buffer before each one (the call launches kernels only: no memset, no host
synchronisation, so it records cleanly). Cases: the 2-D bubble (launch-bound,
where the graph pays) and a 3-D case with the ghost cells read in place and
the signal speed reduced by the last stage."""
import numpy as np
import pytest
import torch

import paper_1901_02955_amd as snap
import workloads as wl
from tests import cases as C

pytestmark = pytest.mark.gpu

CFL = 0.9
STEPS = 5


@pytest.mark.parametrize("name", ["2d_bubble_64x64", "3d_smooth_35x21x19"])
def test_steps_cfl_graph_replays_match_eager(name):
    c = C.build_case(name, dict(C.SPECS)[name])
    g = c.grid
    print(f"[graph] {name}", flush=True)
    dg = snap.device_grid(g)
    work = snap.workspace(dg, snap.SNAP_OP_RK3_CFL)
    states = [torch.as_tensor(c.q).cuda()]
    for seed in (61, 62):
        s = states[0].clone()
        gi = g.interior(s)
        gi[0] += 1e-4 * torch.as_tensor(wl.seeded_normal(gi[0].shape, seed)).cuda() * gi[0].abs().max()
        states.append(s)
    eager = []
    for s in states:
        a = s.clone()
        snap.snap_rk3_steps_cfl(dg, a, CFL, STEPS, work)
        eager.append(g.interior(a).clone())
    torch.cuda.synchronize()
    qd = states[0].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        snap.snap_rk3_steps_cfl(dg, qd, CFL, STEPS, work)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        snap.snap_rk3_steps_cfl(dg, qd, CFL, STEPS, work)
    torch.cuda.synchronize()
    for rnd in range(2):
        for i, s in enumerate(states):
            qd.copy_(s)
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(g.interior(qd), eager[i]), (rnd, i)
            # eager work on the same workspace between replays
            b = s.clone()
            snap.snap_rk3_steps_cfl(dg, b, CFL, STEPS, work)
            torch.cuda.synchronize()
            assert torch.equal(g.interior(b), eager[i]), (rnd, i)
    snap.snap_rk3_steps_status(dg, work)
    del graph
