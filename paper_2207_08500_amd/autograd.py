"""torch.autograd.Function wrappers around the hand-written backward kernels.

* ClassifierBCE: mean binary cross entropy of the classifier over a batch of
  raw six-point stencils (eq. Crossentropy); its backward is the library's
  classifier gradient kernel (FP32 vector units or BF16 MFMA), not torch.
* AdvectionRHS: right-hand side of the advection equation at fixed candidate
  masks (a linear map of u once the selection is fixed); its backward is the
  library's adjoint kernel neno6_rhs_adjoint.
* RHSFixedLabels: right-hand side of the Burgers or 1D Euler equations with
  the labels held fixed (a smooth function of the state away from ties in
  the Rusanov speed); its backward is the library's vector-Jacobian kernel
  neno6_rhs_vjp (through the fluxes, the Roe average and the eigenvectors).

Only argument marshalling happens here; every arithmetic step runs in
libneno6.so.
"""
from __future__ import annotations

import torch

from . import native


class ClassifierBCE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, s: torch.Tensor, y: torch.Tensor,
                precision: int = native.FP32):
        grad = torch.empty_like(params)
        loss = torch.empty(1, dtype=torch.float64, device=params.device)
        native.neno6_classifier_grad(params.detach().contiguous(), s.contiguous(), y.contiguous(),
                                     precision, grad, loss)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return grad * gout, None, None, None


class AdvectionRHS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, masks: torch.Tensor, prob: "native.Problem"):
        if prob.equation != native.ADVECTION or prob.selector != native.SEL_MASKS_IN:
            raise ValueError("AdvectionRHS needs an advection problem with SEL_MASKS_IN")
        rhs = torch.empty_like(u)
        native.neno6_rhs(prob, None, u.detach().contiguous(), rhs, prob.workspace(u.device),
                         masks_in=masks)
        ctx.prob = prob
        ctx.save_for_backward(masks)
        return rhs

    @staticmethod
    def backward(ctx, rbar):
        (masks,) = ctx.saved_tensors
        ubar = torch.empty_like(rbar)
        native.neno6_rhs_adjoint(ctx.prob, masks, rbar.contiguous(), ubar)
        return ubar, None, None


class RHSFixedLabels(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q: torch.Tensor, masks: torch.Tensor, prob: "native.Problem"):
        if prob.equation not in (native.BURGERS, native.EULER1D, native.EULER2D) or \
                prob.selector != native.SEL_MASKS_IN:
            raise ValueError("RHSFixedLabels needs a Burgers or Euler problem with SEL_MASKS_IN")
        qd = q.detach().contiguous()
        rhs = torch.empty_like(qd)
        native.neno6_rhs(prob, None, qd, rhs, prob.workspace(q.device), masks_in=masks)
        ctx.prob = prob
        ctx.save_for_backward(qd, masks)
        return rhs

    @staticmethod
    def backward(ctx, rbar):
        qd, masks = ctx.saved_tensors
        qbar = torch.empty_like(qd)
        native.neno6_rhs_vjp(ctx.prob, qd, masks, rbar.contiguous(), qbar)
        return qbar, None, None


def classifier_bce(params, s, y, precision=native.FP32):
    return ClassifierBCE.apply(params, s, y, precision)


def advection_rhs(u, masks, prob):
    return AdvectionRHS.apply(u, masks, prob)


def rhs_fixed_labels(q, masks, prob):
    return RHSFixedLabels.apply(q, masks, prob)
