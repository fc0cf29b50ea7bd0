"""Parity cases beyond the products: the stored near field entry by entry,
ACA blocks of the workgroup classes (256 and 1,024 threads) against the exact
blocks, a partition with 65-column dense blocks, tied Morton keys, and 48
geometries in one handle against each geometry's exact rows."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from gpu_util import leaf_table_from_gpu, node_rounding_tol, rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# element-wise relative tolerance of a stored entry: FP64 evaluation is the
# oracle's rule up to the rounding of the node positions (node_rounding_tol,
# at least 1e-14); FP32 rounds the centroid difference to float and sums
# seven float reciprocal square roots
ENTRY_TOL = {"f64": 1e-14, "f32": 2e-6, "f16": 2e-6}


def _check_dense(H, op, blocks, prec, count=None, seed=0):
    perm = H.perm()
    idx = np.arange(len(blocks))
    if count is not None and count < len(blocks):
        idx = np.random.default_rng(seed).choice(len(blocks), count, replace=False)
    worst = 0.0
    for b in idx:
        r0, r1, c0, c1 = blocks[b, :4]
        D = H.dense_entries(int(b), blocks)
        ref = op.block(perm[r0:r1], perm[c0:c1])
        dev = np.abs(D - ref) / np.abs(ref)
        tol = ENTRY_TOL[prec]
        if prec == "f64":
            ii, jj = np.meshgrid(perm[r0:r1], perm[c0:c1], indexing="ij")
            tol = node_rounding_tol(op, ii, jj, floor=tol)
        assert np.all(dev <= tol), (b, float(dev.max()))
        worst = max(worst, float(np.max(dev / tol)))
    return worst


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dense_entries_every_block_n1280(oracle_ops, ico, prec):
    import paper_1806_11558_amd as hm
    V, T = ico(3)
    op, _ = oracle_ops(3)
    say("dense entries N = 1280", prec)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec)
    db = H.dense_blocks()
    assert len(db) > 0
    w = _check_dense(H, op, db, prec)
    say("worst dense entry deviation over its tolerance", w)
    assert H.stats()["dense_entries"] == int(((db[:, 1] - db[:, 0]) * (db[:, 3] - db[:, 2])).sum())
    H.free()


@pytest.fixture(scope="module")
def l6():
    from oracle import bem
    from synthetic import icosphere
    V, T = icosphere(6)
    return V, T, bem.Operator(V, T)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_dense_entries_sampled_n81920(l6, prec):
    import paper_1806_11558_amd as hm
    V, T, op = l6
    say("dense entries N = 81920", prec)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=1e-6 if prec != "f16" else 1e-4,
                   max_rank=64, precision=prec)
    _check_dense(H, op, H.dense_blocks(), prec, count=200, seed=3)
    H.free()


@pytest.mark.parametrize("cls", ["wg256", "wg1024"])
@pytest.mark.parametrize("prec,eps", [("f64", 1e-6), ("f32", 1e-6), ("f64", 1e-8)])
def test_aca_workgroup_classes_vs_exact(prec, eps, cls):
    """16 blocks of each workgroup class against their exact blocks:
    256 < max(m, n) <= 4096 (one 256-thread workgroup per block) on the
    icosphere L=6 and max(m, n) > 4096 (one 1,024-thread workgroup per block;
    the smallest such blocks, 5,120 x 5,120) on L=7, leaf 64, eta 1."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere
    level = 6 if cls == "wg256" else 7
    V, T = icosphere(level)
    op = bem.Operator(V, T)
    say("aca", cls, prec, eps, "N =", T.shape[0])
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=eps, max_rank=64, precision=prec)
    lb = H.lr_blocks()
    mx = np.maximum(lb[:, 1] - lb[:, 0], lb[:, 3] - lb[:, 2])
    if cls == "wg256":
        pool = np.flatnonzero((mx > 256) & (mx <= 4096))
    else:
        pool = np.flatnonzero(mx > 4096)
        pool = pool[mx[pool] == mx[pool].min()]
    assert pool.size >= 16
    picks = np.random.default_rng(4).choice(pool, 16, replace=False)
    # the factors come from the device here; the exact blocks in threads
    facs = {int(b): H.lr_factors(int(b)) for b in picks}
    perm = H.perm()
    H.free()

    def one(b):
        r0, r1, c0, c1 = lb[b, :4]
        U, Vf = facs[int(b)]
        Ab = op.block(perm[r0:r1], perm[c0:c1])
        return float(np.linalg.norm(Ab - U @ Vf.T) / np.linalg.norm(Ab))

    with ThreadPoolExecutor(8) as ex:
        errs = list(ex.map(one, picks))
    say("worst", max(errs), "ranks", sorted(set(lb[picks, 4].tolist())))
    assert max(errs) <= 10 * eps, errs


def _mesh65():
    from synthetic import icosphere
    V, T = icosphere(4)
    keep = np.sort(np.random.default_rng(3).choice(T.shape[0], 516, replace=False))
    return V, T[keep]


@pytest.mark.parametrize("prec,eps,bound", [("f64", 1e-8, 1e-7), ("f32", 1e-6, 1e-5)])
def test_dense_blocks_wider_than_64(prec, eps, bound):
    """N = 516 with leaf 64: sibling clusters of 64 and 65 points, so dense
    blocks of 64 x 65 and 65 x 64 entries reach the near-field kernel's path
    for more than 64 columns."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import normal_columns
    V, T = _mesh65()
    op = bem.Operator(V, T)
    A = op.dense()
    say("65-column dense blocks", prec)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=eps, precision=prec)
    db = H.dense_blocks()
    n = db[:, 3] - db[:, 2]
    assert (n > 64).any()
    _check_dense(H, op, db, prec)
    X = normal_columns(op.n, 3, seed=6)
    for vec in ("f64", "f32"):
        xt = torch.tensor(X, device=DEV, dtype=torch.float64 if vec == "f64" else torch.float32)
        Y = H.matvec(xt).double().cpu().numpy()
        YT = H.matvec_T(xt).double().cpu().numpy()
        b = bound + (1e-6 if vec == "f32" else 0.0)
        for k in range(3):
            assert rel2(Y[:, k], A @ X[:, k]) <= b
            assert rel2(YT[:, k], A.T @ X[:, k]) <= b
    H.free()


@pytest.mark.parametrize("leaf", [32, 7])
def test_tied_morton_keys(leaf):
    """Near-duplicate triangles (moved by 1e-7): dozens of Morton keys tie,
    and the sort must keep tied triangles in their original order."""
    import paper_1806_11558_amd as hm
    from oracle import bem, cluster
    from synthetic import icosphere, normal_columns, with_near_duplicates
    V, T = with_near_duplicates(*icosphere(3), count=60, shift=1e-7, seed=5)
    C = bem.centroids(V, T.astype(np.int64))
    P = cluster.Partition(C, leaf, 1.0)
    _, cnt = np.unique(P.keys, return_counts=True)
    assert (cnt > 1).sum() >= 20
    say("tied keys leaf", leaf, "tied groups", int((cnt > 1).sum()))
    H = hm.HMatrix(V, T, leaf_size=leaf, eta=1.0, eps=1e-8, precision="f64")
    assert np.array_equal(H.morton_keys(), P.keys)
    assert np.array_equal(H.perm(), P.perm.astype(np.int32))
    cl = H.clusters()
    assert np.array_equal(cl[:, 0], P.lo) and np.array_equal(cl[:, 1], P.hi)
    assert np.array_equal(H.boxes(), P.boxes)
    assert np.array_equal(leaf_table_from_gpu(H), P.leaf_table())
    # the product still matches the dense operator (entries of the
    # near-duplicate pairs are large but finite)
    A = bem.Operator(V, T).dense()
    x = normal_columns(T.shape[0], 1, seed=7)[:, 0]
    y = H.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    assert rel2(y, A @ x) <= 1e-7
    H.free()


def test_batch48_sampled_rows():
    """48 seeded perturbed spheres (seed g, icosphere level 4 + g mod 3;
    N = 1,720,320 in one handle), FP32 form at ACA eps 1e-5 with the
    autotuned product schedule: 8 right-hand sides (seeds 1000 + g), 24
    sampled rows of every geometry against its exact rows, each column within
    10 eps."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import normal_columns, perturbed_sphere, sample_rows
    eps = 1e-5
    meshes = [perturbed_sphere(4 + g % 3, seed=g) for g in range(48)]
    sizes = [t.shape[0] for _, t in meshes]
    X = np.concatenate([normal_columns(k, 8, seed=1000 + g) for g, k in enumerate(sizes)])
    say("batch48 N =", int(sum(sizes)))
    H = hm.HMatrix.batch(meshes, leaf_size=64, eta=1.0, eps=eps, max_rank=64, precision="f32",
                         autotune=True)
    assert H.stats()["n_geom"] == 48 and H.stats()["cap_hits"] == 0
    off = H.offsets
    ys = {}
    for vec in ("f64", "f32"):
        xt = torch.tensor(X, device=DEV, dtype=torch.float64 if vec == "f64" else torch.float32)
        ys[vec] = (H.matvec(xt).double().cpu().numpy(), H.matvec_T(xt).double().cpu().numpy())
    H.free()

    def one(g):
        V, T = meshes[g]
        op = bem.Operator(V, T)
        rows = sample_rows(T.shape[0], 24, seed=2000 + g)
        a = off[g]
        Xg = X[a:a + T.shape[0]]
        return rows, op.matvec_rows(Xg, rows), op.rmatvec_cols(Xg, rows)

    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(one, range(48)))
    worst = 0.0
    for g, (rows, yr, yc) in enumerate(refs):
        a = off[g]
        for vec, (Y, YT) in ys.items():
            for k in range(8):
                e = max(rel2(Y[a + rows, k], yr[:, k]), rel2(YT[a + rows, k], yc[:, k]))
                worst = max(worst, e)
                assert e <= 10 * eps, (g, vec, k, e)
    say("batch48 worst sampled error", worst)
