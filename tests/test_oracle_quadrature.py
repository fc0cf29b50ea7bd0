"""Pins of the oracle's quadrature and entries against closed forms and
independent integration (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import bem, quadrature


def _rule_on_reference(fun):
    # reference triangle (0,0), (1,0), (0,1): area 1/2
    v0, v1, v2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    y = quadrature.nodes(v0, v1, v2)
    return 0.5 * float(np.sum(quadrature.WEIGHTS * fun(y[:, 0], y[:, 1])))


@pytest.mark.parametrize("a,b", [(a, b) for a in range(6) for b in range(6) if a + b <= 5])
def test_radon_rule_exact_to_degree_5(a, b):
    # int_T x^a y^b = a! b! / (a + b + 2)! on the reference triangle
    exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
    got = _rule_on_reference(lambda x, y: x ** a * y ** b)
    assert abs(got - exact) <= 1e-15 * max(1.0, exact) + 1e-17


def test_radon_rule_not_exact_at_degree_6():
    exact = math.factorial(6) / math.factorial(8)
    got = _rule_on_reference(lambda x, y: x ** 6)
    assert abs(got - exact) > 1e-6


def test_weights_and_barycentrics():
    assert abs(quadrature.WEIGHTS.sum() - 1.0) < 1e-15
    assert np.allclose(quadrature.BARY.sum(axis=1), 1.0, atol=1e-15)
    assert (quadrature.BARY > 0).all()


def test_self_term_equilateral_closed_form():
    # centroid of an equilateral triangle of side s: int 1/|x-y| = sqrt(3) s ln(2 + sqrt(3))
    for s in (1.0, 0.37, 2.5e-3):
        v0 = np.array([[0.0, 0.0, 0.0]])
        v1 = np.array([[s, 0.0, 0.0]])
        v2 = np.array([[s / 2, s * math.sqrt(3) / 2, 0.0]])
        x = (v0 + v1 + v2) / 3
        got = bem.self_integral(x, v0, v1, v2)[0]
        exact = math.sqrt(3.0) * s * math.log(2.0 + math.sqrt(3.0))
        assert abs(got - exact) <= 1e-13 * exact


def _polar_self_integral(x, v0, v1, v2):
    """int_T 1/|x-y| by adaptive quadrature in polar coordinates about x:
    for each sub-triangle (x, a, b), int dphi int_0^{r(phi)} dr."""
    total = 0.0
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        def r_edge(t):
            p = a + t * (b - a)
            return p
        # parametrise the edge by t and integrate the polar angle element
        # dphi = |(p - x) x dp/dt| / |p - x|^2 dt, radial integral = |p - x|
        def integrand(t):
            p = r_edge(t) - x
            dp = b - a
            cr = np.linalg.norm(np.cross(p, dp))
            return cr / np.linalg.norm(p)
        val, _ = integrate.quad(integrand, 0.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)
        total += val
    return total


@pytest.mark.parametrize("seed", range(5))
def test_self_term_general_triangles_vs_adaptive(seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, 3))
    x = (v[0] + v[1] + v[2]) / 3
    got = bem.self_integral(x[None], v[0][None], v[1][None], v[2][None])[0]
    ref = _polar_self_integral(x, v[0], v[1], v[2])
    assert abs(got - ref) <= 1e-10 * ref


def _exact_panel_integral(x, v0, v1, v2):
    """int_T 1/(4 pi |x - y|) dsigma_y by nested adaptive quadrature."""
    e1, e2 = v1 - v0, v2 - v0
    area2 = np.linalg.norm(np.cross(e1, e2))

    def f(t, s):
        y = v0 + s * e1 + t * e2
        return 1.0 / np.linalg.norm(x - y)
    val, _ = integrate.dblquad(f, 0.0, 1.0, lambda s: 0.0, lambda s: 1.0 - s,
                               epsabs=0, epsrel=1e-12)
    return val * area2 / (4 * math.pi)


def test_offdiagonal_entries_vs_adaptive_integration(oracle_ops):
    op, _ = oracle_ops(2)
    rng = np.random.default_rng(3)
    rows = rng.choice(op.n, 6, replace=False)
    cols = rng.choice(op.n, 6, replace=False)
    vals = op.block(rows, cols)
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            if i == j:
                continue
            T = op.T[j]
            exact = _exact_panel_integral(op.x[i], op.V[T[0]], op.V[T[1]], op.V[T[2]])
            d = np.linalg.norm(op.x[i] - op.x[j])
            h = math.sqrt(op.area[j])
            # degree-5 rule: relative error ~ (h/d)^6 for separated panels
            tol = 5e-2 * (h / d) ** 6 + 1e-13
            assert abs(vals[a, b] - exact) <= tol * abs(exact), (i, j, d / h)


def test_diagonal_uses_self_term(oracle_ops):
    op, _ = oracle_ops(2)
    idx = np.arange(0, op.n, 17)
    assert np.array_equal(np.diag(op.block(idx, idx)), op.diag[idx])


def test_kernel_symmetry(oracle_ops):
    op, _ = oracle_ops(3)
    rng = np.random.default_rng(4)
    rows = rng.choice(op.n, 12, replace=False)
    cols = rng.choice(op.n, 12, replace=False)
    A1 = op.block(rows, cols)
    A2 = op.block(cols, rows).T
    # a_ij / |T_j| and a_ji / |T_i| both equal G(x_i, x_j) up to O((h/d)^2)
    checked = 0
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            d = np.linalg.norm(op.x[i] - op.x[j])
            h = max(np.sqrt(op.area[i]), np.sqrt(op.area[j]))
            if d > 5 * h:
                u, v = A1[a, b] / op.area[j], A2[a, b] / op.area[i]
                assert abs(u - v) <= (h / d) ** 2 * u
                checked += 1
    assert checked > 20
    # G(x, y) = G(y, x) bitwise: (x - y)^2 is exact under negation
    x = op.x[5]
    y = op.y[40, 3]
    g1 = 1.0 / np.sqrt(np.sum((x - y) ** 2))
    g2 = 1.0 / np.sqrt(np.sum((y - x) ** 2))
    assert g1 == g2
