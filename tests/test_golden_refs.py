"""The stored full-size references (tests/golden/*_L8_refs.npz) against the
live oracle: a few of their rows and columns recomputed here must agree, so
a stored file cannot drift from the oracle it was written by.  CPU only."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def l8():
    from synthetic import icosphere, mesh_sha256
    V, T = icosphere(8)
    return V, T, mesh_sha256(V, T)


def _load(name, sha):
    g = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    assert str(g["mesh_sha256"]) == sha, "golden file is for another mesh"
    return g


def test_collocation_refs_match_the_oracle(l8):
    from oracle import bem
    from synthetic import normal_columns
    V, T, sha = l8
    g = _load("icosphere_L8_refs.npz", sha)
    X = normal_columns(T.shape[0], g["y"].shape[1], seed=int(g["x_seed"]))
    op = bem.Operator(V, T)
    pick = np.array([0, len(g["rows"]) // 2, len(g["rows"]) - 1])
    idx = g["rows"][pick]
    assert np.allclose(op.matvec_rows(X, idx), g["y"][pick], rtol=1e-12, atol=0)
    assert np.allclose(op.rmatvec_cols(X, idx), g["yT"][pick], rtol=1e-12, atol=0)


def test_galerkin_refs_match_the_oracle(l8):
    from oracle import galerkin
    from synthetic import normal_columns
    V, T, sha = l8
    g = _load("galerkin_icosphere_L8_refs.npz", sha)
    X = normal_columns(T.shape[0], g["y"].shape[1], seed=int(g["x_seed"]))
    op = galerkin.GalerkinOperator(V, T)
    k = len(g["rows"]) // 3
    i = int(g["rows"][k])
    assert np.allclose(op.matvec_rows(X, [i])[0], g["y"][k], rtol=1e-12, atol=0)
    col = op.block(np.arange(op.n), [i])[:, 0]
    assert np.allclose(col @ X, g["yT"][k], rtol=1e-12, atol=0)
