"""Pins of the Galerkin oracle (Sec. 2.2, eq. linearSystem; Sec. 4.1 and 4.3):
the collapsed Gauss rule against exact monomial integrals, the closed-form
inner integral against the pinned in-plane self-term formula and an
independent Duffy quadrature, the singular entries against adaptive
quadrature, symmetry of the matrix, and the paper's harmonic test on the
unit sphere (interior potential error eps(h) falling at third order)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import bem, galerkin


def _ref_triangle():
    return np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


@pytest.mark.parametrize("q", [2, 4, 6])
def test_collapsed_rule_exact_to_degree_2q_minus_2(q):
    T = _ref_triangle()
    pts, w = galerkin.collapsed_rule(T[0], T[1], T[2], q)
    assert abs(w.sum() - 0.5) < 1e-15
    for a in range(2 * q - 1):
        for b in range(2 * q - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = float(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b))
            assert abs(got - exact) <= 1e-14 * max(1.0, exact), (a, b)


def _duffy_inner(x, v0, v1, v2, q):
    """Independent brute force for int_T dsigma_y / |x - y|: T split at the
    projection x' of x into signed triangles, each integrated numerically in
    collapsed coordinates with the collapsed corner at x' (converges slowly
    where x' nears an edge, fast elsewhere)."""
    n = np.cross(v1 - v0, v2 - v0)
    nh = n / np.linalg.norm(n)
    xp = x - np.dot(x - v0, nh) * nh
    g, w = np.polynomial.legendre.leggauss(q)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    s, t = np.meshgrid(g, g, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    s, t, wgt = s.ravel(), t.ravel(), (ws * wt).ravel()
    total = 0.0
    for b, c in ((v0, v1), (v1, v2), (v2, v0)):
        jac = float(np.dot(np.cross(b - xp, c - b), nh))
        y = xp[None, :] + s[:, None] * (b - xp)[None, :] + (s * t)[:, None] * (c - b)[None, :]
        total += jac * float(np.sum(wgt * s / np.linalg.norm(x[None, :] - y, axis=1)))
    return total


def test_inner_integral_in_plane_matches_self_term_formula():
    rng = np.random.default_rng(0)
    for _ in range(5):
        T = rng.standard_normal((3, 3))
        u, v = rng.random(2)
        if u + v > 1:
            u, v = 1 - u, 1 - v
        x = T[0] + u * (T[1] - T[0]) + v * (T[2] - T[0])
        ref = bem.self_integral(x[None], T[0][None], T[1][None], T[2][None])[0]
        assert abs(galerkin.inner_integral(x, *T) - ref) <= 1e-13 * abs(ref)


def test_inner_integral_off_plane_matches_brute_force():
    rng = np.random.default_rng(1)
    T = rng.standard_normal((3, 3))
    c = T.mean(axis=0)
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n /= np.linalg.norm(n)
    pts = [c + 0.3 * n, c + 2.0 * rng.standard_normal(3), T[0] + 0.05 * n + 0.1 * (T[1] - T[0]),
           c - 0.01 * n, T[1] + 0.5 * (T[1] - c)]           # last one: in plane, outside T
    for x in pts:
        ref = _duffy_inner(x, *T, 200)
        assert abs(galerkin.inner_integral(x, *T) - ref) <= 1e-10 * abs(ref), x


def test_inner_integral_far_point_matches_seven_point_rule():
    from oracle import quadrature
    T = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.03, 0.08, 0.02]])
    area = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
    y = quadrature.nodes(T[0], T[1], T[2])
    for d in (1.0, 3.0):
        x = np.array([0.2, -0.4, d])
        rule = area * float(np.sum(quadrature.WEIGHTS / np.linalg.norm(x - y, axis=1)))
        got = galerkin.inner_integral(x, *T)
        assert abs(got - rule) <= (0.15 / d) ** 6 * abs(got)


def _adaptive_entry(Ti, Tj):
    """a_ij by adaptive 2-D quadrature over T_i of the closed-form inner
    integral (scipy dblquad; independent of the collapsed Gauss rule)."""
    e1, e2 = Ti[1] - Ti[0], Ti[2] - Ti[0]
    jac = np.linalg.norm(np.cross(e1, e2))

    def f(v, u):
        return galerkin.inner_integral(Ti[0] + u * e1 + v * e2, *Tj)
    val, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=1e-10, epsrel=1e-7)
    return val * jac / (4.0 * math.pi)


def test_identical_equilateral_entry_vs_adaptive_quadrature():
    T = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, math.sqrt(3.0) / 2.0, 0.0]])
    ref = _adaptive_entry(T, T)
    got = galerkin.entry_singular(T, T)
    # the outer 12 x 12 rule meets the logarithmic edge behaviour of the inner
    # integral: 3.1e-5 relative on this triangle
    assert abs(got - ref) <= 5e-5 * ref


def test_touching_pairs_vs_adaptive_quadrature(ico):
    V, T = ico(1)
    op = galerkin.GalerkinOperator(V, T)
    i = 0
    tri = set(T[i].tolist())
    edge = next(j for j in range(1, op.n) if len(tri & set(T[j].tolist())) == 2)
    vert = next(j for j in range(1, op.n) if len(tri & set(T[j].tolist())) == 1)
    for j in (edge, vert):
        ref = _adaptive_entry(op.tri(i), op.tri(j))
        got = galerkin.entry_singular(op.tri(i), op.tri(j))
        assert abs(got - ref) <= 2e-5 * abs(ref), j


def test_far_entry_matches_singular_rule_of_distant_pair():
    # two distant triangles: the 7 x 7 rule and the outer-Gauss + closed-form
    # rule are two different quadratures of the same smooth integral
    Ti = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0]])
    Tj = Ti + np.array([0.7, 0.2, 0.4])
    a, b = galerkin.entry_far(Ti, Tj), galerkin.entry_singular(Ti, Tj)
    assert abs(a - b) <= (0.1 / 0.8) ** 6 * abs(b)


def test_matrix_symmetric_to_quadrature_accuracy(ico):
    V, T = ico(2)
    A = galerkin.GalerkinOperator(V, T).dense()
    assert np.abs(A - A.T).max() <= 5e-5 * np.abs(A).max()
    # far entries are exactly symmetric (same products in swapped order)
    far = np.abs(A - A.T) <= 1e-15 * np.abs(A)
    assert far.mean() > 0.9


def test_interior_error_third_order_on_the_unit_sphere(ico):
    """Sec. 4.3: f = 4 x1^2 - 3 x2^2 - x3^2 is the trace of a harmonic
    function, so the single-layer potential of the Galerkin density must
    reproduce f inside; eps(h) over interior points falls at third order."""
    rng = np.random.default_rng(3)
    P = rng.standard_normal((100, 3))
    P *= (0.7 * rng.random(100) ** (1.0 / 3.0) / np.linalg.norm(P, axis=1))[:, None]

    def f(y):
        return 4.0 * y[..., 0] ** 2 - 3.0 * y[..., 1] ** 2 - y[..., 2] ** 2
    eps = []
    for level in (1, 2, 3):
        V, T = ico(level)
        op = galerkin.GalerkinOperator(V, T)
        s = np.linalg.solve(op.dense(), op.rhs(f))
        eps.append(float(np.max(np.abs(galerkin.potential(V, T, s, P) - f(P)))))
    assert eps[0] > eps[1] > eps[2]
    assert math.log2(eps[1] / eps[2]) >= 2.5 and math.log2(eps[0] / eps[1]) >= 2.5
    assert eps[2] < 1e-3
