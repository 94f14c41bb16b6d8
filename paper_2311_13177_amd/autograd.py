"""The lifted forward model as a differentiable torch operation.

``LiftedForward.apply(vol, plan, y)`` returns M_b . DFT2(P_b vol) - M_b . y_b for every
blade (Section 4.2 of the paper) through ``vp_forward``; its backward applies the
hand-written adjoint ``vp_adjoint`` (mask, unitary inverse DFT, transposed shear
gather), so ``loss.backward()`` yields dL/dRe + i dL/dIm of the volume, torch's
convention for complex parameters. ``BladeAlignedForward`` does the same for samples on
each blade's rotated lattice (the gridding operators). Both directions run on the
caller's current stream; torch only provides the memory.
"""

from __future__ import annotations

import torch

from . import binding as B


class LiftedForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vol: torch.Tensor, plan: "B.Plan", y: torch.Tensor | None = None) -> torch.Tensor:
        ctx.plan = plan
        return B.vp_forward(plan, vol.contiguous(), None if y is None else y.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        grad = B.vp_adjoint(ctx.plan, grad_out.contiguous())
        return grad, None, None


class Regulariser(torch.autograd.Function):
    """Identity in the forward pass; its backward adds the TV/L1 gradient of the volume.

    Use as ``vol_r = Regulariser.apply(vol, plan, tv_weight, l1_weight, tv_eps)`` and
    build the data term on ``vol_r``: the gradient reaching ``vol`` is then the data
    gradient plus tv_weight * grad TV + l1_weight * grad L1 (Section 4.3).
    """

    @staticmethod
    def forward(ctx, vol, plan, tv_weight: float, l1_weight: float, tv_eps: float):
        ctx.save_for_backward(vol)
        ctx.args = (plan, float(tv_weight), float(l1_weight), float(tv_eps))
        return vol.view_as(vol)

    @staticmethod
    def backward(ctx, grad_out):
        (vol,) = ctx.saved_tensors
        plan, tv_w, l1_w, eps = ctx.args
        grad = grad_out.contiguous().clone()
        B.vp_tv_grad(plan, vol.contiguous(), tv_w, l1_w, eps, grad, accumulate=True)
        return grad, None, None, None, None


class BladeAlignedForward(torch.autograd.Function):
    """The lifted model sampled on each blade's own rotated lattice (``vp_nu_forward``,
    samples [B][Lmax][n], lines beyond a blade's count zero) minus y; its backward is the
    exact transpose ``vp_nu_adjoint`` (padding lines of the incoming gradient ignored)."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, plan: "B.Plan", y: torch.Tensor | None = None) -> torch.Tensor:
        ctx.plan = plan
        return B.vp_nu_forward(plan, vol.contiguous(), None if y is None else y.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        return B.vp_nu_adjoint(ctx.plan, grad_out.contiguous()), None, None


def blade_aligned_forward(vol: torch.Tensor, plan: "B.Plan", y: torch.Tensor | None = None) -> torch.Tensor:
    return BladeAlignedForward.apply(vol, plan, y)


def lifted_forward(vol: torch.Tensor, plan: "B.Plan", y: torch.Tensor | None = None) -> torch.Tensor:
    return LiftedForward.apply(vol, plan, y)

