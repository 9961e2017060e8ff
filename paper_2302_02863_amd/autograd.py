"""Differentiable solve u = A_h(s, kappa)^{-1} F for PyTorch (argument marshalling only).

Forward builds the operator for the given nodal fields and solves with
``fpde_solve``; backward solves the adjoint system A_h lambda = dJ/du (A_h is
symmetric) with the same CG and returns, through ``fpde_apply_adjoint`` with
scale alpha = -1,

    dJ/ds     = -grad_s(lambda, u),   dJ/dkappa = -grad_kappa(lambda, u),   dJ/dF = lambda,

since A_h du = -(dA_h) u for fixed F.  Every step runs in libfpde's kernels.
The operator lives as long as the autograd context, so a graph kept with
``retain_graph=True`` can be differentiated again.
"""
from __future__ import annotations

import torch

from .operator import Operator


class FracSolve(torch.autograd.Function):
    """u = FracSolve.apply(s, kappa, F, mesh, opts, rtol) for s, kappa [F, n_nodes] and F [F, N, R] or [F, N].

    u has the shape of F.
    """

    @staticmethod
    def forward(ctx, s, kappa, F, mesh, opts, rtol=1e-12):
        op = Operator(mesh, s.detach().to("cpu", torch.float64).numpy(),
                      kappa.detach().to("cpu", torch.float64).numpy(), opts)
        Fd = F.detach().to(torch.float64).contiguous()
        u, _ = op.solve(Fd, rtol=rtol)
        ctx.op = op          # freed with the context (Operator.__del__ releases the device memory)
        ctx.rtol = rtol
        ctx.where = ((s.device, s.dtype), (kappa.device, kappa.dtype), (F.device, F.dtype))
        ctx.save_for_backward(u)
        return u.reshape(F.shape).to(F.dtype)

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        op = ctx.op
        lam, _ = op.solve(gu.detach().to(torch.float64).reshape(u.shape).contiguous(), rtol=ctx.rtol)
        gs, gk = op.apply_adjoint(lam, u, alpha=-1.0)
        (ds, ts), (dk, tk), (df, tf) = ctx.where
        return gs.to(ds, ts), gk.to(dk, tk), lam.reshape(gu.shape).to(df, tf), None, None, None


def frac_solve(s, kappa, F, mesh, opts, rtol=1e-12):
    return FracSolve.apply(s, kappa, F, mesh, opts, rtol)


__all__ = ["FracSolve", "frac_solve"]
