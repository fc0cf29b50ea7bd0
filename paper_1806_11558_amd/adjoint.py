"""Differentiable solve: sigma = H^{-1} f with dJ/df = H^{-T} dJ/dsigma.

Both directions call the library's GMRES (hm_solve); the backward pass solves
the adjoint system with the transposed H-matrix product.  The Function only
marshals arguments."""
from __future__ import annotations

import torch


class HSolve(torch.autograd.Function):
    """sigma = HSolve.apply(f, H, tol, restart, max_iter)."""

    @staticmethod
    def forward(ctx, f, H, tol=1e-10, restart=100, max_iter=2000):
        sigma, info, status = H.solve(f.contiguous(), tol=tol, restart=restart,
                                      max_iter=max_iter)
        ctx.H, ctx.tol, ctx.restart, ctx.max_iter = H, tol, restart, max_iter
        ctx.info = info
        return sigma

    @staticmethod
    def backward(ctx, g):
        lam, info, status = ctx.H.solve(g.contiguous(), tol=ctx.tol, restart=ctx.restart,
                                        max_iter=ctx.max_iter, transpose=True)
        return lam, None, None, None, None


def hsolve(f, H, tol=1e-10, restart=100, max_iter=2000):
    return HSolve.apply(f, H, tol, restart, max_iter)
