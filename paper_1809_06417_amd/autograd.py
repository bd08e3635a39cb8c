"""Differentiable render: torch.autograd.Function over the hand-written
forward march and adjoint (reverse) march of librte.

The backward recomputes the transmittance in a reverse march from the
per-ray exit optical depth (FP64) saved by the forward; the in-scatter grid is held
fixed (no gradient flows into it).
"""
from __future__ import annotations

import torch

from .rte import Plan

__all__ = ["RenderFunction", "render"]


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: Plan, emission, extinction, inscatter=None):
        emission = emission.contiguous()
        extinction = extinction.contiguous()
        images, exit_tau = plan.render_forward(emission, extinction, inscatter)
        ctx.plan = plan
        ctx.save_for_backward(emission, extinction, exit_tau)
        ctx.inscatter = inscatter
        return images

    @staticmethod
    def backward(ctx, grad_images):
        emission, extinction, exit_tau = ctx.saved_tensors
        g_em, g_sig = ctx.plan.render_backward(emission, extinction, ctx.inscatter, exit_tau,
                                               grad_images.contiguous())
        return None, g_em, g_sig, None


def render(plan: Plan, emission, extinction, inscatter=None):
    """Images [V, C, H, W] differentiable w.r.t. emission and extinction."""
    if not plan.gradients:
        raise ValueError("the plan must be created with gradients=True")
    return RenderFunction.apply(plan, emission, extinction, inscatter)
