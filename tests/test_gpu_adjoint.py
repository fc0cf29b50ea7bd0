"""Adjoint of the solve (dJ/df through the transposed H-matrix product):
central finite differences and the dense oracle gradient."""
import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gradient_vs_dense_oracle_and_fd(prec, oracle_ops):
    import paper_1806_11558_amd as hm
    from synthetic import perturbed_sphere
    from oracle import bem
    say("adjoint", prec)
    V, T = perturbed_sphere(3, seed=7)            # N = 1280
    op = bem.Operator(V, T)
    A = op.dense()
    n = op.n
    eps = 1e-8 if prec == "f64" else 1e-6
    H = hm.HMatrix(V, T, leaf_size=32, eps=eps, precision=prec)
    rng = np.random.default_rng(7)
    fstar = rng.standard_normal(n)
    sig_star = torch.tensor(np.linalg.solve(A, fstar), device=DEV)
    f0 = np.random.default_rng(8).standard_normal(n)
    f = torch.tensor(f0, device=DEV, requires_grad=True)
    sigma = hm.hsolve(f, H, tol=1e-11)
    J = 0.5 * torch.sum((sigma - sig_star) ** 2)
    J.backward()
    g = f.grad.cpu().numpy()
    # dense oracle gradient: A^{-T} (A^{-1} f - sigma*)
    g_ref = np.linalg.solve(A.T, np.linalg.solve(A, f0) - sig_star.cpu().numpy())
    kappa = np.linalg.cond(A)
    assert rel2(g, g_ref) <= kappa * 20 * eps
    # central finite differences on random unit directions (J is quadratic in f,
    # so the difference quotient is exact up to the solve tolerance)
    dirs = np.random.default_rng(9).standard_normal((8, n))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    h = 1e-3

    def Jof(fv):
        s = hm.hsolve(torch.tensor(fv, device=DEV), H, tol=1e-12)
        return 0.5 * float(torch.sum((s - sig_star) ** 2))
    for d in dirs:
        fd = (Jof(f0 + h * d) - Jof(f0 - h * d)) / (2 * h)
        an = float(g @ d)
        # the difference quotient carries the solve error kappa * tol * |sigma| / h
        assert abs(fd - an) <= 1e-4 * np.linalg.norm(g), (fd, an)
    H.free()


def test_gradient_vs_dense_oracle_n5120_fp32():
    """Perturbed sphere seed 7 at N = 5,120, FP32 form, leaf 64: the adjoint
    gradient against the dense oracle's A^{-T}(A^{-1} f - sigma*)."""
    import paper_1806_11558_amd as hm
    from synthetic import perturbed_sphere
    from oracle import bem
    say("adjoint dense N=5120 f32")
    V, T = perturbed_sphere(4, seed=7)
    op = bem.Operator(V, T)
    A = op.dense()
    n = op.n
    eps = 1e-6
    H = hm.HMatrix(V, T, leaf_size=64, eps=eps, precision="f32")
    fstar = np.random.default_rng(7).standard_normal(n)
    sig_star = np.linalg.solve(A, fstar)
    f0 = np.random.default_rng(8).standard_normal(n)
    f = torch.tensor(f0, device=DEV, requires_grad=True)
    sigma = hm.hsolve(f, H, tol=1e-10)
    J = 0.5 * torch.sum((sigma - torch.tensor(sig_star, device=DEV)) ** 2)
    J.backward()
    g = f.grad.cpu().numpy()
    H.free()
    g_ref = np.linalg.solve(A.T, np.linalg.solve(A, f0) - sig_star)
    kappa = np.linalg.cond(A)                 # about 163
    assert rel2(g, g_ref) <= kappa * 20 * eps


def test_gradient_fd_n81920_fp32():
    """Perturbed sphere seed 7 at N = 81,920, FP32 form, leaf 64: dJ/df for
    J = 1/2 |sigma - sigma*|^2, sigma* = H^{-1} f*, against central
    differences (h = 1e-3) on 64 seeded unit directions."""
    import paper_1806_11558_amd as hm
    from synthetic import perturbed_sphere
    say("adjoint fd N=81920 f32")
    V, T = perturbed_sphere(6, seed=7)
    n = T.shape[0]
    H = hm.HMatrix(V, T, leaf_size=64, eps=1e-6, precision="f32")
    fstar = torch.tensor(np.random.default_rng(7).standard_normal(n), device=DEV)
    sig_star = hm.hsolve(fstar, H, tol=1e-11).detach()
    f0 = np.random.default_rng(8).standard_normal(n)
    f = torch.tensor(f0, device=DEV, requires_grad=True)
    sigma = hm.hsolve(f, H, tol=1e-11)
    J = 0.5 * torch.sum((sigma - sig_star) ** 2)
    J.backward()
    g = f.grad.cpu().numpy()
    dirs = np.random.default_rng(9).standard_normal((64, n))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    h = 1e-3

    def Jof(fv):
        s = hm.hsolve(torch.tensor(fv, device=DEV), H, tol=1e-11)
        return 0.5 * float(torch.sum((s - sig_star) ** 2))
    gn = np.linalg.norm(g)
    worst = 0.0
    for d in dirs:
        fd = (Jof(f0 + h * d) - Jof(f0 - h * d)) / (2 * h)
        worst = max(worst, abs(fd - float(g @ d)) / gn)
    H.free()
    # J is quadratic in f: the quotient is exact up to the solve tolerance
    assert worst <= 1e-4, worst
