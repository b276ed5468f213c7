"""Reverse-mode differentiation of the N-1 branch-overload screening loss.

``OverloadLoss`` wraps ``gpcg_overload_gradients`` of the device library in a
``torch.autograd.Function``: the forward pass returns the loss of every
outage scenario, L_j = sum_e softplus(kappa (|f_e| / F_e - 1)) on the flows
of the re-dispatched post-outage solution (Section IV); the backward pass
recomputes the angles, runs one adjoint PCG per scenario with the same
base-case ILU(0) preconditioner, and contracts the per-scenario gradients
with the incoming weights (``gpcg_weighted_rows``).  Marshalling only: every
step runs in the library's kernels.
"""
from __future__ import annotations

import torch


class OverloadLoss(torch.autograd.Function):
    """loss[j] = L_j(P, x) for the outages given; differentiable in P and x.

    ``x`` must hold the reactances the context was built with (the context's
    matrix and factors belong to them); it is an input so that autograd
    tracks the dependence.  ``F`` (flow limits) is a constant.
    """

    @staticmethod
    def forward(fctx, P, x, context, outages, F, kappa=20.0, tol=1e-12, max_iter=20000):
        out = context.overload_gradients(outages, P, F, kappa, tol, max_iter, grads=False)
        fctx.context = context
        fctx.args = (kappa, tol, max_iter)
        fctx.save_for_backward(P, outages, F)
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_loss):
        P, outages, F = fctx.saved_tensors
        kappa, tol, max_iter = fctx.args
        ctx = fctx.context
        out = ctx.overload_gradients(outages, P, F, kappa, tol, max_iter, grads=True)
        w = grad_loss.contiguous().to(torch.float64)
        gP = torch.empty(ctx.n_bus, dtype=torch.float64, device=P.device)
        gx = torch.empty(ctx.m, dtype=torch.float64, device=P.device)
        ctx.weighted_rows(out["grad_p"], w, gP)
        ctx.weighted_rows(out["grad_x"], w, gx)
        return gP, gx, None, None, None, None, None, None


def overload_loss(P, x, context, outages, F, kappa=20.0, tol=1e-12, max_iter=20000):
    """Per-scenario overload loss, differentiable in P and x."""
    return OverloadLoss.apply(P, x, context, outages, F, kappa, tol, max_iter)
