"""Several meshes in one handle (hm_build_batch): per-geometry Morton keys,
permutations and block partitions bit-exact against the oracle run on each
mesh alone; products and solves against the block-diagonal dense operator;
every geometry's share equal to a handle built on that mesh alone."""
import numpy as np
import pytest
import torch

from gpu_util import leaf_table_from_gpu, rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _meshes():
    from synthetic import icosphere, perturbed_sphere
    V0, T0 = icosphere(2)                         # 320
    V1, T1 = perturbed_sphere(3, seed=1)          # 1280
    V2, T2 = icosphere(3)                         # 1280, shifted and subset
    V2 = V2 * 0.5 + np.array([3.0, -1.0, 0.5])
    keep = np.sort(np.random.default_rng(5).choice(T2.shape[0], 1000, replace=False))
    return [(V0, T0), (V1, T1), (V2, T2[keep])]


@pytest.fixture(scope="module")
def batch():
    import paper_1806_11558_amd as hm
    from oracle import bem
    meshes = _meshes()
    H = hm.HMatrix.batch(meshes, leaf_size=32, eta=1.0, eps=1e-8, precision="f64")
    ops = [bem.Operator(V, T) for V, T in meshes]
    yield meshes, H, ops
    H.free()


def test_batch_structure_bit_exact(batch):
    from oracle import bem, cluster
    meshes, H, ops = batch
    say("batch structure")
    off = H.offsets
    assert H.stats()["n_geom"] == len(meshes)
    keys, perm = H.morton_keys(), H.perm()
    tabs, cls = [], []
    for g, (V, T) in enumerate(meshes):
        C = bem.centroids(V, T.astype(np.int64))
        P = cluster.Partition(C, 32, 1.0)
        a, b = off[g], off[g + 1]
        assert np.array_equal(keys[a:b], P.keys)
        assert np.array_equal(perm[a:b], (P.perm + a).astype(np.int32))
        t = P.leaf_table().copy()
        t[:, :4] += a
        tabs.append(t)
        cls.append(np.c_[P.lo + a, P.hi + a, P.level])
    ref = np.concatenate(tabs)
    ref = ref[np.lexsort(ref.T[::-1])]
    assert np.array_equal(leaf_table_from_gpu(H), ref)
    got = H.clusters()
    got = np.c_[got[:, 0], got[:, 1], got[:, 3]]
    exp = np.concatenate(cls)
    assert np.array_equal(got[np.lexsort(got.T[::-1])], exp[np.lexsort(exp.T[::-1])])


def test_batch_products_and_solve(batch):
    from synthetic import normal_columns
    meshes, H, ops = batch
    say("batch products")
    off = H.offsets
    X = normal_columns(H.n, 8, seed=0)             # 8 right-hand sides per geometry
    xt = torch.tensor(X, device=DEV)
    Y = H.matvec(xt).cpu().numpy()
    YT = H.matvec_T(xt).cpu().numpy()
    dense = [op.dense() for op in ops]
    for g, A in enumerate(dense):
        a, b = off[g], off[g + 1]
        for k in range(8):
            assert rel2(Y[a:b, k], A @ X[a:b, k]) <= 1e-7
            assert rel2(YT[a:b, k], A.T @ X[a:b, k]) <= 1e-7
    F = np.ones((H.n, 8)) + 0.1 * X
    sig, info, status = H.solve(torch.tensor(F, device=DEV), tol=1e-10)
    assert status == 0
    S = sig.cpu().numpy()
    for g, A in enumerate(dense):
        a, b = off[g], off[g + 1]
        ref = np.linalg.solve(A, F[a:b])
        assert rel2(S[a:b], ref) <= np.linalg.cond(A) * 1e-7


def test_batch_equals_single_builds(batch):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    meshes, H, ops = batch
    say("batch vs single")
    off = H.offsets
    X = normal_columns(H.n, 3, seed=4)
    Y = H.matvec(torch.tensor(X, device=DEV)).cpu().numpy()
    for g, (V, T) in enumerate(meshes):
        a, b = off[g], off[g + 1]
        Hg = hm.HMatrix(V, T, leaf_size=32, eta=1.0, eps=1e-8, precision="f64")
        yg = Hg.matvec(torch.tensor(X[a:b], device=DEV)).cpu().numpy()
        Hg.free()
        assert rel2(Y[a:b], yg) <= 1e-13
