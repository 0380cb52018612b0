"""Differentiable multi-step SSP-RK3 integration on the GPU (torch.autograd).

``rk3_run(grid, q0, dt, nsteps, checkpoint_every)`` advances a padded state by
``nsteps`` calls of ``snap_rk3_step`` and, under autograd, back-propagates
through them with ``snap_rk3_step_adjoint`` (the discrete adjoint of the
three-stage scheme of Sec. 4.3 with fixed dt). Memory is bounded by step
checkpointing: the forward pass keeps the state every ``checkpoint_every``
steps; the backward pass re-runs each segment from its checkpoint, keeping the
segment's states, and then walks it in reverse. With ``keep_stages`` (the
default) the re-run also keeps every step's two stage states, so that the
adjoint step does not recompute them (``snap_rk3_step_adjoint_stages``): a
segment then holds three padded states per step instead of one. The forward
pass keeps the last segment that way already, so the backward pass starts
without a re-run.

``kessler_step(grid, q, dt, kessler)`` is the Kessler microphysics step
(Sec. 3, ``snap_kessler_step``) under autograd, back-propagated with
``snap_kessler_step_adjoint``; it composes with ``rk3_run`` for operator-split
dynamics and microphysics. ``saturation_adjust(grid, q, adjust)`` is the
saturation adjustment (App. D, ``snap_saturation_adjust``) the same way, with
``snap_saturation_adjust_adjoint``.

Only the interior of the state carries gradients: the library overwrites ghost
layers from the interior on every call, so the gradient with respect to the
ghost layers of ``q0`` is zero, and ghost layers of the output (unspecified
after a step) receive no gradient.
"""
from __future__ import annotations

import torch

from . import (SNAP_NG, SNAP_OP_RK3, SNAP_OP_RK3_ADJ, DeviceGrid, SnapKesslerC, SnapSatAdjC,
               kessler_params, satadj_params, snap_kessler_step, snap_kessler_step_adjoint,
               snap_rk3_step, snap_rk3_step_adjoint, snap_rk3_step_adjoint_stages,
               snap_saturation_adjust, snap_saturation_adjust_adjoint, workspace)


def _interior(grid: DeviceGrid, q: torch.Tensor) -> torch.Tensor:
    g = SNAP_NG
    gy = grid.gy
    return q[:, g:g + grid.nz, gy:gy + grid.ny, g:g + grid.nx]


class _SnapRK3Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q0: torch.Tensor, grid: DeviceGrid, dt: float, nsteps: int,
                checkpoint_every: int, keep_stages: bool):
        work = workspace(grid, SNAP_OP_RK3)
        q = q0.detach().clone()
        checkpoints = []
        last = (nsteps - 1) // checkpoint_every * checkpoint_every   # first step of the last segment
        kept_states, kept_stages = [], []
        for n in range(nsteps):
            if n % checkpoint_every == 0:
                checkpoints.append(q.clone())
            if keep_stages and n >= last:
                # the last segment: its states and stage states, as the backward re-run keeps them
                kept_states.append(q.clone())
                kept_stages.append(workspace(grid, SNAP_OP_RK3))
                snap_rk3_step(grid, q, dt, kept_stages[-1])
            else:
                snap_rk3_step(grid, q, dt, work)
        ctx.grid, ctx.dt, ctx.nsteps, ctx.every = grid, dt, nsteps, checkpoint_every
        ctx.keep_stages = keep_stages
        ctx.checkpoints = checkpoints
        ctx.last_segment = (kept_states, kept_stages) if keep_stages else None
        return q

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        grid, dt, nsteps, every = ctx.grid, ctx.dt, ctx.nsteps, ctx.every
        work = workspace(grid, SNAP_OP_RK3)
        awork = workspace(grid, SNAP_OP_RK3_ADJ)
        qbar = _interior(grid, grad_out).contiguous().clone()
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            start = seg * every
            stop = min(start + every, nsteps)
            if ctx.keep_stages and seg == len(ctx.checkpoints) - 1:
                states, stages = ctx.last_segment
                ctx.last_segment = None
                for t in range(stop - start - 1, -1, -1):
                    snap_rk3_step_adjoint_stages(grid, states[t], stages[t], dt, qbar, awork)
                del stages, states
                continue
            states = [ctx.checkpoints[seg].clone()]
            if ctx.keep_stages:
                # every step of the segment, the last included, for its stage states
                stages = []
                for t in range(start, stop):
                    stages.append(workspace(grid, SNAP_OP_RK3))
                    nxt = states[-1].clone()
                    snap_rk3_step(grid, nxt, dt, stages[-1])
                    if t < stop - 1:
                        states.append(nxt)
                for t in range(stop - start - 1, -1, -1):
                    snap_rk3_step_adjoint_stages(grid, states[t], stages[t], dt, qbar, awork)
                del stages
            else:
                for _ in range(start, stop - 1):
                    nxt = states[-1].clone()
                    snap_rk3_step(grid, nxt, dt, work)
                    states.append(nxt)
                for t in range(stop - start - 1, -1, -1):
                    snap_rk3_step_adjoint(grid, states[t], dt, qbar, awork)
            del states
        grad_in = torch.zeros_like(grad_out)
        _interior(grid, grad_in).copy_(qbar)
        ctx.checkpoints = None
        ctx.last_segment = None
        return grad_in, None, None, None, None, None


def rk3_run(grid: DeviceGrid, q0: torch.Tensor, dt: float, nsteps: int,
            checkpoint_every: int = 20, keep_stages: bool = True) -> torch.Tensor:
    """State after ``nsteps`` SSP-RK3 steps of fixed ``dt``; differentiable in q0's interior.

    keep_stages: keep the stage states of a segment's steps for the backward
    pass (three padded states per step of a segment) instead of recomputing
    them in every adjoint step (one per step).
    """
    if nsteps < 1 or checkpoint_every < 1:
        raise ValueError("nsteps and checkpoint_every must be >= 1")
    return _SnapRK3Run.apply(q0, grid, float(dt), int(nsteps), int(checkpoint_every),
                             bool(keep_stages))


class _SnapKesslerStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q: torch.Tensor, grid: DeviceGrid, dt: float, params):
        q0 = q.detach().clone()
        out = q0.clone()
        snap_kessler_step(grid, out, dt, params)
        ctx.grid, ctx.dt, ctx.params = grid, dt, params
        ctx.save_for_backward(q0)
        return out

    @staticmethod
    def backward(ctx, g_out: torch.Tensor):
        (q0,) = ctx.saved_tensors
        grid = ctx.grid
        qb = _interior(grid, g_out).contiguous().clone()
        snap_kessler_step_adjoint(grid, q0, ctx.dt, ctx.params, qb)
        g_in = torch.zeros_like(g_out)
        _interior(grid, g_in).copy_(qb)
        return g_in, None, None, None


def kessler_step(grid: DeviceGrid, q: torch.Tensor, dt: float, kessler) -> torch.Tensor:
    """Padded state after one Kessler microphysics step of length dt, differentiable
    with respect to ``q`` (the step's adjoint, within the interior)."""
    params = kessler if isinstance(kessler, SnapKesslerC) else kessler_params(kessler)
    return _SnapKesslerStep.apply(q, grid, dt, params)


class _SnapSaturationAdjust(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q: torch.Tensor, grid: DeviceGrid, params):
        q0 = q.detach().clone()
        out = q0.clone()
        snap_saturation_adjust(grid, out, params)
        ctx.grid, ctx.params = grid, params
        ctx.save_for_backward(q0)
        return out

    @staticmethod
    def backward(ctx, g_out: torch.Tensor):
        (q0,) = ctx.saved_tensors
        grid = ctx.grid
        qb = _interior(grid, g_out).contiguous().clone()
        snap_saturation_adjust_adjoint(grid, q0, ctx.params, qb)
        g_in = torch.zeros_like(g_out)
        _interior(grid, g_in).copy_(qb)
        return g_in, None, None


def saturation_adjust(grid: DeviceGrid, q: torch.Tensor, adjust) -> torch.Tensor:
    """Padded state after the saturation adjustment, differentiable with respect
    to ``q`` (the adjustment's adjoint, within the interior)."""
    params = adjust if isinstance(adjust, SnapSatAdjC) else satadj_params(adjust)
    return _SnapSaturationAdjust.apply(q, grid, params)
