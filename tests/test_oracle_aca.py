"""Pins of the oracle's ACA (Sec. 2.3) against exact low-rank blocks, the SVD
(Eckart-Young) and the interpolation property."""
import numpy as np
import pytest

from oracle import aca, cluster


@pytest.mark.parametrize("r", [1, 2, 5, 9])
def test_exact_rank_blocks_stop_at_rank(r):
    rng = np.random.default_rng(r)
    A = rng.standard_normal((50, r)) @ rng.standard_normal((r, 37))
    U, V = aca.aca_dense(A, 1e-12)
    # the stopping test is applied to the term just kept: after the r exact
    # terms at most one more term of rounding size is taken
    assert U.shape[1] in (r, r + 1)
    if U.shape[1] == r + 1:
        assert np.linalg.norm(U[:, r]) * np.linalg.norm(V[:, r]) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(A - U @ V.T) <= 1e-12 * np.linalg.norm(A)


def test_zero_block_has_rank_zero():
    U, V = aca.aca_dense(np.zeros((7, 5)), 1e-6)
    assert U.shape == (7, 0) and V.shape == (5, 0)


def test_zero_rows_are_skipped():
    A = np.zeros((6, 4))
    A[3] = [1.0, -2.0, 0.5, 0.0]
    U, V = aca.aca_dense(A, 1e-14)
    assert U.shape[1] == 1 and np.allclose(U @ V.T, A)


def test_fixed_rank_mode():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 30))
    U, V = aca.aca_dense(A, 0.0, 7)
    assert U.shape[1] == 7


def test_pivots_reproduce_rows_and_columns():
    # cross approximation interpolates the pivot rows and columns
    rng = np.random.default_rng(2)
    x = rng.random((40, 3))
    y = rng.random((30, 3)) + np.array([3.0, 0, 0])
    A = 1.0 / np.linalg.norm(x[:, None] - y[None], axis=-1)
    U, V = aca.aca_dense(A, 1e-8)
    R = A - U @ V.T
    piv_cols = [int(np.argmax(np.abs(V[:, l]) == 1.0)) for l in range(V.shape[1])]
    for j in piv_cols:
        assert np.abs(R[:, j]).max() <= 1e-12 * np.abs(A).max()


def test_blocks_of_the_operator_vs_svd(oracle_ops):
    """Real admissible blocks: error <= 10 eps; the rank is at least the
    Eckart-Young rank needed for the achieved error and not far above the
    SVD rank at eps."""
    op, _ = oracle_ops(4)
    P = cluster.Partition(op.x, 64, 1.0)
    rng = np.random.default_rng(0)
    idx = rng.choice(np.flatnonzero(P.adm), 12, replace=False)
    for eps in (1e-4, 1e-6):
        for b in idx:
            rows = P.perm[P.lo[P.t[b]]:P.hi[P.t[b]]]
            cols = P.perm[P.lo[P.s[b]]:P.hi[P.s[b]]]
            A = op.block(rows, cols)
            U, V = aca.aca_dense(A, eps, 64)
            err = np.linalg.norm(A - U @ V.T) / np.linalg.norm(A)
            assert err <= 10 * eps
            sv = np.linalg.svd(A, compute_uv=False)
            tail = np.sqrt(np.cumsum((sv ** 2)[::-1]))[::-1] / np.linalg.norm(sv)
            need = int(np.argmax(tail <= err)) if (tail <= err).any() else sv.size
            assert U.shape[1] >= need
            r_svd = int(np.argmax(tail <= eps)) if (tail <= eps).any() else sv.size
            assert U.shape[1] <= 2 * r_svd + 3
