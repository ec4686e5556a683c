"""The trajectory cost as a torch.autograd.Function: the forward pass runs the kinematics, sphere
cost and aggregation kernels, the backward pass the hand-written adjoint kernel (Sec. III-B steps
(2)-(5)).  The workspace holding the stored tensors is kept from forward to backward."""
from __future__ import annotations

import torch

from .context import Context, Shape


class VaprCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q: torch.Tensor, vctx: Context, shape: Shape):
        cost, ws = vctx.cost_fwd(q.detach().contiguous(), shape)
        ctx.save_for_backward(q, ws)
        ctx.vctx = vctx
        return cost

    @staticmethod
    def backward(ctx, grad_cost: torch.Tensor):
        q, ws = ctx.saved_tensors
        up = grad_cost.detach().to(torch.float64).contiguous()
        grad_q = ctx.vctx.cost_bwd(q.detach().contiguous(), ws, up)
        return grad_q, None, None


def trajectory_cost(q: torch.Tensor, vctx: Context, shape: Shape) -> torch.Tensor:
    """Differentiable trajectory-candidate costs [shape.n_tc] (float64) of configurations q [B, 7]."""
    return VaprCost.apply(q, vctx, shape)
