"""Closed forms on the unit sphere: the discrete operator converges to the
continuous single-layer operator (pins of the oracle operator as a whole)."""
import numpy as np
import pytest

from oracle import bem, sphere


def _errors(oracle_ops, levels, fn):
    out = []
    for L in levels:
        op, A = oracle_ops(L, dense=True)
        out.append(fn(op, A))
    return np.array(out)


def test_constant_density_has_unit_potential(oracle_ops):
    # S 1 = 1 on the unit sphere: the solution of A s = 1 tends to 1
    errs = _errors(oracle_ops, (2, 3, 4), lambda op, A: np.abs(np.linalg.solve(A, np.ones(op.n)) - 1).max())
    assert errs[-1] < 5e-3
    rates = errs[:-1] / errs[1:]
    assert (rates > 1.8).all(), errs        # first order in h (halving h halves the error)


def test_matvec_of_constant_is_one(oracle_ops):
    errs = _errors(oracle_ops, (2, 3, 4), lambda op, A: np.abs(A @ np.ones(op.n) - 1).max())
    assert errs[-1] < 1e-2 and (errs[:-1] / errs[1:] > 1.8).all(), errs


@pytest.mark.parametrize("l", [1, 2, 3])
def test_spherical_harmonics_are_eigenfunctions(oracle_ops, l):
    # V Y_l = Y_l / (2l + 1)
    def err(op, A):
        y = sphere.zonal_harmonic(l, op.x)
        return np.abs(A @ y - y / (2 * l + 1)).max() / np.abs(y).max()
    errs = _errors(oracle_ops, (2, 3, 4), err)
    assert (errs[:-1] / errs[1:] > 1.7).all(), errs
    assert errs[-1] < 1e-2


def test_paper_rhs_density_and_interior_solution(oracle_ops):
    # f = 4x^2 - 3y^2 - z^2 is harmonic; on the unit sphere sigma = 5 f and the
    # single-layer potential reproduces f inside (the paper's error measure)
    rng = np.random.default_rng(0)
    pts = rng.standard_normal((20, 3))
    pts *= (0.5 * rng.random(20) ** (1 / 3) / np.linalg.norm(pts, axis=1))[:, None]
    dens, interior = [], []
    for L in (2, 3, 4):
        op, A = oracle_ops(L, dense=True)
        xn = op.x / np.linalg.norm(op.x, axis=1)[:, None]
        f = sphere.paper_rhs(op.x)
        s = bem.solve_dense(A, f)
        dens.append(np.abs(s - 5 * sphere.paper_rhs(xn)).max())
        interior.append(np.abs(op.potential(s, pts) - sphere.paper_rhs(pts)).max())
    dens, interior = np.array(dens), np.array(interior)
    assert (dens[:-1] / dens[1:] > 1.6).all(), dens
    assert (interior[:-1] / interior[1:] > 1.6).all(), interior
    assert interior[-1] < 1e-2


def test_dense_solve_is_a_solution(oracle_ops):
    op, A = oracle_ops(3, dense=True)
    f = np.random.default_rng(1).standard_normal(op.n)
    s = bem.solve_dense(A, f)
    assert np.linalg.norm(A @ s - f) <= 1e-12 * np.linalg.norm(f) * np.linalg.cond(A)


def test_golden_discretisation_errors(oracle_ops):
    """Regression against values written by tests/golden/make_golden.py
    (oracle only); the values themselves are calibrated, not printed by the
    paper (parity unpinned for the exact numbers)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "sphere_errors.json")
    gold = json.load(open(path))
    for key, val in gold["constant_density_maxerr"].items():
        op, A = oracle_ops(int(key), dense=True)
        got = np.abs(np.linalg.solve(A, np.ones(op.n)) - 1).max()
        assert abs(got - val) <= 1e-9 * val
