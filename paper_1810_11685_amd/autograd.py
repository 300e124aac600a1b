"""torch.autograd.Functions over the acoustic operator, with hand-written
backward passes.

* `acoustic(p0, plan)` maps p0 to sensor data H_a p0; its backward is the
  adjoint solve H_a^* (Lemma 2).  H_a is linear in p0 and the transposed
  one-step map T^* does not depend on the forward state (Section 3.2.4), so
  this backward needs no stored wavefield and the function keeps none.
* `acoustic_medium(p0, c0, plan, ckpt_interval=K)` maps (p0, c0) to the same
  data and differentiates in the sound speed too.  That gradient correlates
  the forward wavefield with the adjoint one, so the backward recomputes the
  forward in reverse from checkpoints of the stacked state taken every K
  iterates (memory O(nt/K + K) instead of O(nt)), through qpat_medium_grad.
  c0 must be the sound speed the plan was built from (the plan holds the
  medium tables; a different c0 needs a new plan).

`replay_states` exposes the same checkpoint facility directly: it recomputes
any segment of forward states from a checkpoint buffer.
"""
from __future__ import annotations

import numpy as np
import torch

from .ops import Plan


class AcousticForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0: torch.Tensor, plan: Plan):
        ctx.plan = plan
        return plan.forward(p0.detach())

    @staticmethod
    def backward(ctx, grad_data: torch.Tensor):
        g = ctx.plan.adjoint(grad_data.contiguous()) if ctx.needs_input_grad[0] else None
        return g, None


def acoustic(p0: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Sensor data H_a p0 ([..., nt, ns]); differentiable in p0."""
    return AcousticForward.apply(p0, plan)


class AcousticMediumForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0: torch.Tensor, c0: torch.Tensor, plan: Plan, ckpt_interval: int | None):
        c_plan = plan.sound_speed()
        if tuple(c0.shape) != c_plan.shape or not np.array_equal(c0.detach().double().cpu().numpy(), c_plan):
            raise ValueError("acoustic_medium: c0 must be the sound speed the plan was built from")
        ctx.plan = plan
        ctx.interval = ckpt_interval
        ctx.save_for_backward(p0.detach())
        return plan.forward(p0.detach())

    @staticmethod
    def backward(ctx, grad_data: torch.Tensor):
        (p0,) = ctx.saved_tensors
        gc, gp = ctx.plan.medium_grad(p0, grad_data.contiguous(), interval=ctx.interval)
        if p0.dim() > 2:              # one c0 for every vector of the batch
            gc = gc.reshape(-1, *gc.shape[-2:]).sum(0)
        return (gp if ctx.needs_input_grad[0] else None,
                gc.double() if ctx.needs_input_grad[1] else None, None, None)


def acoustic_medium(p0: torch.Tensor, c0: torch.Tensor, plan: Plan, ckpt_interval: int | None = 100):
    """Sensor data H_a[c0] p0, differentiable in p0 and in the sound speed c0
    ([ny, nx], float64, equal to the plan's).  The c0 gradient recomputes the
    forward wavefield from checkpoints every `ckpt_interval` iterates (None:
    keep every sensitivity)."""
    return AcousticMediumForward.apply(p0, c0, plan, ckpt_interval)


def replay_states(plan: Plan, p0: torch.Tensor, ckpt: torch.Tensor, interval: int):
    """Yield (m0, states) for the segments in reverse order: states[:, c] is z_{m0+c}."""
    nseg = ckpt.shape[1]
    for seg in range(nseg - 1, -1, -1):
        yield seg * interval, plan.replay(p0, ckpt, interval, seg)
