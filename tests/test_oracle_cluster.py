"""Pins of the oracle's clustering and block partition (Sec. 2.3, Sec. 3.1,
Algorithm 1) against hand examples, brute force and invariants."""
import numpy as np
import pytest

from oracle import bem, cluster


def _brute_morton(C):
    """Independent Morton keys: quantise, write the 21-bit binary strings and
    interleave them character by character (x first)."""
    a = C.min(axis=0)
    ext = (C.max(axis=0) - a).max()
    keys = []
    for p in C:
        q = [min(int(np.floor((p[d] - a[d]) * (2.0 ** 21 / ext))), 2 ** 21 - 1) for d in range(3)]
        s = [format(v, "021b") for v in q]
        keys.append(int("".join(s[0][k] + s[1][k] + s[2][k] for k in range(21)), 2))
    return np.array(keys, dtype=np.uint64)


def test_morton_unit_cube_corners():
    # corners of a cube: with x as the most significant bit of every triple,
    # the corners sort as (0,0,0), (0,0,1), (0,1,0), ..., (1,1,1)
    corners = np.array([[x, y, z] for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)])
    rng = np.random.default_rng(0)
    shuffled = corners[rng.permutation(8)]
    order = cluster.morton_order(cluster.morton_keys(shuffled))
    assert np.array_equal(shuffled[order], corners)
    k = cluster.morton_keys(corners)
    assert k[0] == 0 and k[-1] == (1 << 63) - 1


def test_morton_against_string_interleave():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((300, 3)) * np.array([1.0, 0.3, 2.0])
    assert np.array_equal(cluster.morton_keys(C), _brute_morton(C))


def test_morton_sort_is_stable():
    C = np.array([[0.5, 0.5, 0.5]] * 4 + [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    order = cluster.morton_order(cluster.morton_keys(C))
    assert list(order) == [4, 0, 1, 2, 3, 5]


@pytest.mark.parametrize("n,leaf", [(1280, 32), (81920, 64), (1000, 7), (33, 32), (1, 32), (65, 64)])
def test_cluster_tree_properties(n, leaf):
    lo, hi, child, level = cluster.cluster_tree(n, leaf)
    assert lo[0] == 0 and hi[0] == n                                   # (C2)
    assert (hi > lo).all()                                             # (C1)
    is_leaf = child < 0
    assert (hi[is_leaf] - lo[is_leaf] <= leaf).all()                   # (C3)
    for k in np.flatnonzero(~is_leaf):                                 # (C4) + CBC balance
        c1, c2 = child[k], child[k] + 1
        assert lo[c1] == lo[k] and hi[c1] == lo[c2] and hi[c2] == hi[k]
        s1, s2 = hi[c1] - lo[c1], hi[c2] - lo[c2]
        assert s1 <= s2 <= s1 + 1
        assert hi[k] - lo[k] > leaf
    # leaves tile [0, n)
    L = np.sort(lo[is_leaf])
    assert L[0] == 0 and np.array_equal(np.sort(hi[is_leaf])[:-1], L[1:])


def test_cluster_depth_for_icosphere_sizes():
    # N = 20 * 4^L halves exactly down to 20 * 4^L / 2^d <= leaf
    for L, leaf, depth, leafsize in ((3, 32, 6, 20), (6, 64, 11, 40), (8, 64, 15, 40)):
        lo, hi, child, level = cluster.cluster_tree(20 * 4 ** L, leaf)
        leaves = child < 0
        assert level.max() == depth
        assert set((hi - lo)[leaves]) == {leafsize}


def test_admissibility_hand_boxes():
    unit = np.array([0.0, 0, 0, 1, 1, 1])
    def shifted(dx):
        return unit + np.array([dx, 0, 0, dx, 0, 0])
    # diam^2 = 3; dist = gap along x
    assert not cluster.admissible(unit, shifted(1.0), 1.0)       # touching: dist 0
    assert not cluster.admissible(unit, shifted(2.0), 1.0)       # gap 1 < sqrt(3)
    assert cluster.admissible(unit, shifted(1.0 + np.sqrt(3.0) + 1e-9), 1.0)
    assert cluster.admissible(unit, shifted(3.0), 1.0)           # gap 2 > sqrt 3
    assert not cluster.admissible(unit, shifted(3.0), 0.5)       # eta = 0.5: sqrt 3 > 0.5 * 2
    assert cluster.admissible(unit, shifted(2.0), 2.0)           # eta = 2: sqrt 3 <= 2 * 1
    # equality counts as admissible: diam^2 = 1 (segment boxes), gap 1, eta 1
    seg = np.array([0.0, 0, 0, 1, 0, 0])
    seg2 = seg + np.array([2.0, 0, 0, 2.0, 0, 0])
    assert cluster.admissible(seg, seg2, 1.0)
    # the smaller box decides (min of diameters)
    big = np.array([-10.0, -10, -10, 0, 0, 0])
    tiny = np.array([1.0, 0, 0, 1.0, 0.0, 0.0])                  # point, diam 0
    assert cluster.admissible(big, tiny, 1.0)
    assert np.isclose(cluster.dist2(big, tiny), 1.0)


def _partition(level, leaf, eta=1.0):
    from synthetic import icosphere
    V, T = icosphere(level)
    return cluster.Partition(bem.centroids(V, T), leaf, eta)


@pytest.mark.parametrize("level,leaf,eta", [(2, 32, 1.0), (3, 32, 1.0), (3, 16, 0.5), (4, 64, 1.0), (3, 7, 2.0)])
def test_partition_characterisation(level, leaf, eta):
    """The leaves of Algorithm 1 are characterised by: (i) they tile I x I,
    (ii) each leaf satisfies the stop condition, (iii) the parent pair of each
    leaf satisfies the split condition.  These three properties determine the
    partition uniquely, so they pin it."""
    P = _partition(level, leaf, eta)
    n = P.lo[0:1].size and P.hi[0]
    t, s, adm = P.t, P.s, P.adm
    m = P.hi[t] - P.lo[t]
    k = P.hi[s] - P.lo[s]
    assert int((m * k).sum()) == n * n
    cover = np.zeros((n, n), dtype=np.int32)
    for a, b in zip(t, s):
        cover[P.lo[a]:P.hi[a], P.lo[b]:P.hi[b]] += 1
    assert (cover == 1).all()
    A = cluster.admissible(P.boxes[t], P.boxes[s], eta)
    assert np.array_equal(A, adm)
    stop = adm | (m <= leaf) | (k <= leaf)
    assert stop.all()
    parent = np.full(P.lo.size, -1)
    for q in np.flatnonzero(P.child >= 0):
        parent[P.child[q]] = q
        parent[P.child[q] + 1] = q
    nonroot = (t != 0) | (s != 0)
    pt, ps = parent[t[nonroot]], parent[s[nonroot]]
    assert (pt >= 0).all() and (ps >= 0).all()
    split = (~cluster.admissible(P.boxes[pt], P.boxes[ps], eta)) & \
        (P.hi[pt] - P.lo[pt] > leaf) & (P.hi[ps] - P.lo[ps] > leaf)
    assert split.all()
    # same level: the block tree only pairs clusters of equal depth
    assert np.array_equal(P.level[t], P.level[s])


def test_partition_symmetric_and_recursive_equals_levelwise():
    P = _partition(3, 32)
    tab = {(a, b, bool(c)) for a, b, c in zip(P.t, P.s, P.adm)}
    assert all((b, a, c) in tab for a, b, c in tab)
    rec = cluster.block_tree_recursive(P.lo, P.hi, P.child, P.boxes, P.eta, P.leaf_size)
    assert {(a, b, bool(c)) for a, b, c in rec} == tab


def test_boxes_contain_members_and_are_tight():
    P = _partition(3, 32)
    for k in range(P.lo.size):
        pts = P.Cs[P.lo[k]:P.hi[k]]
        b = P.boxes[k]
        assert (pts >= b[:3]).all() and (pts <= b[3:]).all()
        assert np.array_equal(pts.min(0), b[:3]) and np.array_equal(pts.max(0), b[3:])


def test_dense_leaves_have_leaf_sizes():
    P = _partition(4, 64)
    m = (P.hi[P.t] - P.lo[P.t])[~P.adm]
    assert set(m.tolist()) == {40}
