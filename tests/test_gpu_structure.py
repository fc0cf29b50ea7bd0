"""Bit-exact parity of the clustering and block partition (GPU vs oracle)."""
import numpy as np
import pytest

from gpu_util import leaf_table_from_gpu, say

pytestmark = pytest.mark.gpu

CASES = [
    ("ico3-leaf32", 3, None, 32, 1.0),
    ("ico6-leaf64", 6, None, 64, 1.0),
    ("ico4-subset1000-leaf7-eta2", 4, 1000, 7, 2.0),
    ("perturbed4-leaf16-eta0.5", "p4", None, 16, 0.5),
    ("ico2-subset33-leaf32", 2, 33, 32, 1.0),
    ("ico0-one-triangle", 0, 1, 32, 1.0),
]


def _mesh(level, subset):
    from synthetic import icosphere, perturbed_sphere
    if level == "p4":
        V, T = perturbed_sphere(4, seed=3)
    else:
        V, T = icosphere(level)
    if subset is not None:
        rng = np.random.default_rng(11)
        T = T[np.sort(rng.choice(T.shape[0], subset, replace=False))]
    return V, T


@pytest.mark.parametrize("name,level,subset,leaf,eta", CASES, ids=[c[0] for c in CASES])
def test_partition_bit_exact(name, level, subset, leaf, eta):
    import paper_1806_11558_amd as hm
    from oracle import bem, cluster
    V, T = _mesh(level, subset)
    say("structure", name, "N =", T.shape[0])
    H = hm.HMatrix(V, T, leaf_size=leaf, eta=eta, eps=1e-4, precision="f64")
    C = bem.centroids(V, T.astype(np.int64))
    P = cluster.Partition(C, leaf, eta)
    assert np.array_equal(H.morton_keys(), P.keys)
    assert np.array_equal(H.perm(), P.perm.astype(np.int32))
    cl = H.clusters()
    # clusters: same breadth-first tree
    assert np.array_equal(cl[:, 0], P.lo) and np.array_equal(cl[:, 1], P.hi)
    assert np.array_equal(cl[:, 2], P.child) and np.array_equal(cl[:, 3], P.level)
    assert np.array_equal(H.boxes(), P.boxes)             # bitwise
    assert np.array_equal(leaf_table_from_gpu(H), P.leaf_table())
    st = H.stats()
    assert st["n_dense"] + st["n_lr"] == len(P.t)
    H.free()
