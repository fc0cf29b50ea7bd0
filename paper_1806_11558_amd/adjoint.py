"""Differentiable solve: sigma = H^{-1} f with dJ/df = H^{-T} dJ/dsigma.

Both directions call the library's GMRES (hm_solve); the backward pass solves
the adjoint system with the transposed H-matrix product.  The Function only
marshals arguments.  A solve that misses its tolerance raises HMError
(status HM_NOT_CONVERGED) instead of returning a wrong density or gradient."""
from __future__ import annotations

import torch

from ._binding import HM_NOT_CONVERGED, HM_OK, HMError


def _checked(H, rhs, what, **kw):
    sigma, info, status = H.solve(rhs.contiguous(), **kw)
    if status != HM_OK:
        raise HMError(HM_NOT_CONVERGED,
                      f"{what} solve did not converge: relative residual {info.rel_residual:.3e} "
                      f"after {info.iters} steps (tol {kw['tol']:g}, max_iter {kw['max_iter']})")
    return sigma


class HSolve(torch.autograd.Function):
    """sigma = HSolve.apply(f, H, tol, restart, max_iter)."""

    @staticmethod
    def forward(ctx, f, H, tol=1e-10, restart=100, max_iter=2000):
        ctx.H, ctx.kw = H, dict(tol=tol, restart=restart, max_iter=max_iter)
        return _checked(H, f, "forward", **ctx.kw)

    @staticmethod
    def backward(ctx, g):
        lam = _checked(ctx.H, g, "adjoint", transpose=True, **ctx.kw)
        return lam, None, None, None, None


def hsolve(f, H, tol=1e-10, restart=100, max_iter=2000):
    return HSolve.apply(f, H, tol, restart, max_iter)
