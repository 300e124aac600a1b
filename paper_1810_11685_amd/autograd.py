"""torch.autograd.Function mapping p0 to sensor data, with the adjoint solve
(Lemma 2) as its hand-written backward.

H_a is linear in p0, so the backward needs no stored wavefield.  With
`ckpt_interval` = K the forward also keeps the stacked state z_m every K steps
(O(nt/K) memory); `replay_states` recomputes any segment from its checkpoint
(O(K) memory) for consumers that need the forward wavefield in reverse order.
"""
from __future__ import annotations

import torch

from .ops import Plan


class AcousticForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0: torch.Tensor, plan: Plan, ckpt_interval: int | None = None):
        if ckpt_interval:
            data, ck = plan.forward_ckpt(p0.detach(), ckpt_interval)
            ctx.ckpt = ck
        else:
            data = plan.forward(p0.detach())
            ctx.ckpt = None
        ctx.plan = plan
        ctx.interval = ckpt_interval
        return data

    @staticmethod
    def backward(ctx, grad_data: torch.Tensor):
        g = ctx.plan.adjoint(grad_data.contiguous()) if ctx.needs_input_grad[0] else None
        return g, None, None


def acoustic(p0: torch.Tensor, plan: Plan, ckpt_interval: int | None = None) -> torch.Tensor:
    """Sensor data H_a p0 ([..., nt, ns]); differentiable in p0."""
    return AcousticForward.apply(p0, plan, ckpt_interval)


def replay_states(plan: Plan, p0: torch.Tensor, ckpt: torch.Tensor, interval: int):
    """Yield (m0, states) for the segments in reverse order: states[:, c] is z_{m0+c}."""
    nseg = ckpt.shape[1]
    for seg in range(nseg - 1, -1, -1):
        yield seg * interval, plan.replay(p0, ckpt, interval, seg)
