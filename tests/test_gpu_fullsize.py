"""Parity at the benchmark's sizes, in the benchmark's configuration (leaf 64,
eta 1, the library's own launch shapes): sampled rows and columns of the
products against the oracle's exact rows and columns, the clustering
bit-exact, and the refined solve to a 1e-8 residual.

Every form is tested at the ACA tolerance it is built for -- eps 1e-6 for the
FP64 and FP32 forms, eps 1e-4 for the FP16-factor form -- and every product
must be within exactly 10 eps of the oracle (the method's bound), with
double and with float vectors.

N = 81,920 (icosphere L=6): 96 rows and columns, computed here by the oracle.
N = 1,310,720 (L=8): 4,096 rows and columns, written by
tests/golden/make_fullsize_refs.py (oracle only); for the Galerkin matrix
256 rows and columns, written by tests/golden/make_galerkin_refs.py (oracle
only).
"""
import os

import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = {"f64": 1e-6, "f32": 1e-6, "f16": 1e-4}
GOLDEN_L8 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "icosphere_L8_refs.npz")
GOLDEN_GAL_L8 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "galerkin_icosphere_L8_refs.npz")


def _vecs(prec):
    return ("f64",) if prec == "f64" else ("f64", "f32")


def _dev(X, vec):
    return torch.tensor(X, device=DEV, dtype=torch.float64 if vec == "f64" else torch.float32)


def _columns_err(y, yref):
    return max(rel2(y[:, k], yref[:, k]) for k in range(yref.shape[1]))


@pytest.fixture(scope="module")
def l6():
    from oracle import bem
    from synthetic import icosphere
    V, T = icosphere(6)
    return V, T, bem.Operator(V, T)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_l6_sampled_products(l6, prec):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns, sample_rows
    V, T, op = l6
    n = op.n
    eps = EPS[prec]
    say("fullsize L6", prec, "eps", eps, "N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=eps, max_rank=64, precision=prec)
    st = H.stats()
    assert st["cap_hits"] == 0
    X = normal_columns(n, 16, seed=0)
    rows = sample_rows(n, 96, seed=1)
    ref = op.matvec_rows(X, rows)
    refT = op.rmatvec_cols(X, rows)
    for vec in _vecs(prec):
        xt = _dev(X, vec)
        y16 = H.matvec(xt).double().cpu().numpy()
        y1 = H.matvec(xt[:, 0].contiguous()).double().cpu().numpy()
        yT16 = H.matvec_T(xt).double().cpu().numpy()
        yT1 = H.matvec_T(xt[:, 0].contiguous()).double().cpu().numpy()
        b = 10 * eps
        assert _columns_err(y16[rows], ref) <= b, vec
        assert rel2(y1[rows], ref[:, 0]) <= b, vec
        assert _columns_err(yT16[rows], refT) <= b, vec
        assert rel2(yT1[rows], refT[:, 0]) <= b, vec
        # one right-hand side and the first of sixteen take different kernels
        agree = 1e-13 if prec == "f64" else 2e-6
        assert rel2(y16[:, 0], y1) <= agree, vec
    H.free()


@pytest.fixture(scope="module")
def l8():
    from synthetic import icosphere, mesh_sha256, normal_columns
    V, T = icosphere(8)
    g = np.load(GOLDEN_L8, allow_pickle=False)
    assert str(g["mesh_sha256"]) == mesh_sha256(V, T), "golden file is for another mesh"
    X = normal_columns(T.shape[0], g["y"].shape[1], seed=int(g["x_seed"]))
    return V, T, X, g["rows"], g["y"], g["yT"]


def _l8_products(H, X, rows, y_ref, yT_ref, eps, vecs):
    errs = {}
    for vec in vecs:
        xt = _dev(X, vec)
        y = H.matvec(xt).double().cpu().numpy()[rows]
        yT = H.matvec_T(xt).double().cpu().numpy()[rows]
        y1 = H.matvec(xt[:, 0].contiguous()).double().cpu().numpy()[rows]
        errs[vec] = (_columns_err(y, y_ref), _columns_err(yT, yT_ref), rel2(y1, y_ref[:, 0]))
        say("L8", vec, "errors (H x, H^T x, 1 rhs):", errs[vec])
        assert max(errs[vec]) <= 10 * eps, (vec, errs[vec])
    return errs


def test_l8_fp32_structure_rows_and_columns(l8):
    import paper_1806_11558_amd as hm
    from oracle import bem, cluster
    V, T, X, rows, y_ref, yT_ref = l8
    n = T.shape[0]
    say("fullsize L8 f32 N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=EPS["f32"], max_rank=64, precision="f32")
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
    _l8_products(H, X, rows, y_ref, yT_ref, EPS["f32"], ("f64", "f32"))
    H.free()


def test_l8_fp64_rows_columns_and_solve(l8):
    """The FP64 form at the full size (the metric's comparison form): 4,096
    exact rows of H x and H^T x within 10 eps, and plain GMRES in double to
    a relative residual of 1e-8, checked again by an independent product."""
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, X, rows, y_ref, yT_ref = l8
    n = T.shape[0]
    eps = EPS["f64"]
    say("fullsize L8 f64 eps", eps, "N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=eps, max_rank=64, precision="f64")
    assert H.stats()["cap_hits"] == 0
    _l8_products(H, X, rows, y_ref, yT_ref, eps, ("f64",))
    f = torch.tensor(normal_columns(n, 1, seed=2)[:, 0], device=DEV)
    say("L8 f64 solve")
    s, info, st = H.solve(f, tol=1e-8, restart=100, max_iter=3000)
    say("L8 f64 solve:", info.iters, "steps, residual", info.rel_residual)
    assert st == hm.HM_OK and info.rel_residual <= 1e-8
    r = f - H.matvec(s)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(f)) <= 1.01e-8
    H.free()
    hm.release_memory()


def test_l8_fp16_rows_columns_and_refined_solve(l8):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, X, rows, y_ref, yT_ref = l8
    n = T.shape[0]
    eps = EPS["f16"]
    say("fullsize L8 f16 eps", eps, "N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=eps, max_rank=64, precision="f16")
    assert H.stats()["cap_hits"] == 0
    _l8_products(H, X, rows, y_ref, yT_ref, eps, ("f64", "f32"))
    # the target solve: FP16 factors, inner GMRES with float products to
    # 1e-4, double refinement to a relative residual of 1e-8
    f = torch.tensor(normal_columns(n, 1, seed=2)[:, 0], device=DEV)
    say("L8 f16 refined solve")
    s, info, st = H.solve(f, tol=1e-8, restart=100, max_iter=3000, refine=True, inner_tol=1e-4)
    say("L8 f16 solve:", info.iters, "steps,", info.ir_steps, "corrections, residual",
        info.rel_residual)
    assert st == hm.HM_OK and info.rel_residual <= 1e-8 and info.ir_steps >= 2
    r = f - H.matvec(s)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(f)) <= 1.01e-8
    H.free()
    hm.release_memory()


def test_l8_galerkin_rows_and_columns():
    """The Galerkin matrix (HM_GALERKIN, FP32, eps 1e-6) at N = 1,310,720:
    H x and H^T x at 256 exact rows and columns of the Galerkin oracle
    within 10 eps, double and float vectors."""
    import paper_1806_11558_amd as hm
    from synthetic import icosphere, mesh_sha256, normal_columns
    V, T = icosphere(8)
    g = np.load(GOLDEN_GAL_L8, allow_pickle=False)
    assert str(g["mesh_sha256"]) == mesh_sha256(V, T), "golden file is for another mesh"
    n = T.shape[0]
    X = normal_columns(n, g["y"].shape[1], seed=int(g["x_seed"]))
    say("fullsize L8 galerkin f32 N =", n)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=EPS["f32"], max_rank=64, precision="f32",
                   operator="galerkin")
    assert H.stats()["cap_hits"] == 0
    _l8_products(H, X, g["rows"], g["y"], g["yT"], EPS["f32"], ("f64", "f32"))
    H.free()
    hm.release_memory()
