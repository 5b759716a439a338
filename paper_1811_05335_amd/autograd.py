"""torch.autograd wrappers around the library's transforms.

NfftFunction       f = A~ fhat with A~ = B(x) F D (the NFFT); gradients with respect to the
                   coefficients (the adjoint NFFT) and to the node positions (window derivative).
InfftApplyFunction fcheck = D^* F^* B_opt^* f (the modified adjoint NFFT, (3.32)); gradient with
                   respect to f is B_opt F D applied to the incoming gradient (Remark 3.24).

B_opt is a constant of the node set it was computed for: the modified adjoint has no gradient with
respect to x, and it runs on its own plan (loading new nodes into a plan invalidates its B_opt).
Gradients follow PyTorch's convention for complex tensors (dL/dx = sum Re(conj(g) df/dx)).
"""
from __future__ import annotations

import torch

from .plan import NfftPlan


class NfftFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan):
        plan.set_nodes(x.detach())
        ctx.plan = plan
        ctx.save_for_backward(fhat)
        return plan.trafo(fhat)

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        (fhat,) = ctx.saved_tensors
        plan = ctx.plan
        g = grad_f.contiguous()
        gfh = plan.adjoint(g) if ctx.needs_input_grad[0] else None
        gx = plan.grad_x(fhat, g) if ctx.needs_input_grad[1] else None
        return gfh, gx, None


class InfftApplyFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, plan: NfftPlan):
        ctx.plan = plan
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_h: torch.Tensor):
        return ctx.plan.apply_adjoint(grad_h.contiguous()), None


def nfft(fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan) -> torch.Tensor:
    """Differentiable NFFT (nodes x are loaded into `plan`)."""
    return NfftFunction.apply(fhat, x, plan)


def infft(f: torch.Tensor, plan: NfftPlan) -> torch.Tensor:
    """Differentiable modified adjoint NFFT with the plan's B_opt (call plan.precompute_B first)."""
    return InfftApplyFunction.apply(f, plan)
