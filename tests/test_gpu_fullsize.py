"""Parity at the benchmark's sizes, in the benchmark's configuration (leaf 64,
eta 1, ACA eps 1e-6, the library's own launch shapes):
sampled rows and columns of the products against the oracle's exact rows and
columns, the clustering bit-exact.

N = 81,920 (icosphere L=6) for the FP64, FP32 and FP16-factor forms with 1
and 16 right-hand sides; N = 1,310,720 (L=8) for the FP32 form with one
right-hand side.
"""
import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = 1e-6
# 10 eps is the product tolerance of the method; the FP32 and FP16 forms add
# their rounding (float accumulation of ~1e3 terms; 2^-11 per FP16 factor
# value relative to its column).
BOUND = {"f64": 10 * EPS, "f32": 10 * EPS + 1e-6, "f16": 10 * EPS + 4 * 2.0 ** -11}


@pytest.fixture(scope="module")
def l6():
    from oracle import bem
    from synthetic import icosphere
    V, T = icosphere(6)
    return V, T, bem.Operator(V, T)


def _columns_err(y, yref):
    return max(rel2(y[:, k], yref[:, k]) for k in range(yref.shape[1]))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_l6_sampled_products(l6, prec):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns, sample_rows
    V, T, op = l6
    n = op.n
    say("fullsize L6", prec, "N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=EPS, max_rank=64, precision=prec)
    st = H.stats()
    assert st["cap_hits"] == 0
    X = normal_columns(n, 16, seed=0)
    rows = sample_rows(n, 96, seed=1)
    ref = op.matvec_rows(X, rows)
    refT = op.rmatvec_cols(X, rows)
    xt = torch.tensor(X, device=DEV)
    y16 = H.matvec(xt).cpu().numpy()
    y1 = H.matvec(xt[:, 0].contiguous()).cpu().numpy()
    yT16 = H.matvec_T(xt).cpu().numpy()
    yT1 = H.matvec_T(xt[:, 0].contiguous()).cpu().numpy()
    H.free()
    b = BOUND[prec]
    assert _columns_err(y16[rows], ref) <= b
    assert rel2(y1[rows], ref[:, 0]) <= b
    assert _columns_err(yT16[rows], refT) <= b
    assert rel2(yT1[rows], refT[:, 0]) <= b
    # one right-hand side and the first of sixteen take different kernels
    assert rel2(y16[:, 0], y1) <= 1e-6 if prec != "f64" else rel2(y16[:, 0], y1) <= 1e-13


def test_l8_fp32_structure_and_rows():
    import paper_1806_11558_amd as hm
    from oracle import bem, cluster
    from synthetic import icosphere, normal_columns, sample_rows
    V, T = icosphere(8)
    n = T.shape[0]
    say("fullsize L8 f32 N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=EPS, max_rank=64, precision="f32")
    C = bem.centroids(V, T.astype(np.int64))
    keys = cluster.morton_keys(C)
    perm = cluster.morton_order(keys)
    assert np.array_equal(H.morton_keys(), keys)
    assert np.array_equal(H.perm(), perm.astype(np.int32))
    lo, hi, child, level = cluster.cluster_tree(n, 64)
    cl = H.clusters()
    assert np.array_equal(cl[:, 0], lo) and np.array_equal(cl[:, 1], hi)
    assert np.array_equal(cl[:, 2], child) and np.array_equal(cl[:, 3], level)
    assert np.array_equal(H.boxes(), cluster.cluster_boxes(C[perm], lo, hi))
    st = H.stats()
    assert st["cap_hits"] == 0 and st["n_leaves"] == 32768
    x = normal_columns(n, 1, seed=0)[:, 0]
    rows = sample_rows(n, 24, seed=1)
    op = bem.Operator(V, T)
    ref = op.matvec_rows(x, rows)
    refT = op.rmatvec_cols(x, rows)
    xt = torch.tensor(x, device=DEV)
    y = H.matvec(xt).cpu().numpy()
    yT = H.matvec_T(xt).cpu().numpy()
    H.free()
    assert rel2(y[rows], ref) <= BOUND["f32"]
    assert rel2(yT[rows], refT) <= BOUND["f32"]
