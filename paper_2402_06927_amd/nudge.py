"""Nudging objective as a differentiable PyTorch function (section 3.1.3).

``NudgeObjective`` maps the controls dLambda [n][n_steps][Q] to the
per-particle objective J = Phi(u^S) - log G [n].  The forward pass calls
``sch_nudge_grad`` once, which also returns dJ/d(dLambda) from the library's
adjoint kernel; the backward pass scales that stored gradient by the incoming
gradient.  No arithmetic of the model runs in PyTorch.
"""
from __future__ import annotations

import torch

from . import sch


class NudgeObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dLambda: torch.Tensor, model: sch.Model, obs: sch.Obs, m0: torch.Tensor,
                u0: torch.Tensor, dW: torch.Tensor | None, ckpt_every: int = 8,
                workspace: torch.Tensor | None = None):
        dLambda = dLambda.detach().contiguous()
        n = dLambda.shape[0]
        J = torch.empty(n, dtype=torch.float64, device=dLambda.device)
        grad = torch.empty_like(dLambda)
        status = torch.empty(n, dtype=torch.int32, device=dLambda.device)
        sch.sch_nudge_grad(model, obs, m0, u0, dW, dLambda, J, grad, ckpt_every, status,
                           workspace)
        ctx.save_for_backward(grad)
        ctx.mark_non_differentiable(status)
        return J, status

    @staticmethod
    def backward(ctx, gJ, _gstatus):
        (grad,) = ctx.saved_tensors
        return gJ.reshape(-1, 1, 1) * grad, None, None, None, None, None, None, None


def nudge_objective(dLambda: torch.Tensor, model: sch.Model, obs: sch.Obs, m0: torch.Tensor,
                    u0: torch.Tensor, dW: torch.Tensor | None = None, ckpt_every: int = 8,
                    workspace: torch.Tensor | None = None):
    """J [n] (differentiable in dLambda) and the per-particle status [n]."""
    return NudgeObjective.apply(dLambda, model, obs, m0, u0, dW, ckpt_every, workspace)
