"""Clustering and block partition, written from Sec. 2.3 and Sec. 3.1.

* Morton codes and sort (Sec. 3.1, "Spatial data structure"): every node of
  X_h gets a Z-order code; sorting by it makes consecutive nodes close, so
  cardinality-based clustering becomes an array decomposition.
  Readings: 21 bits per axis inside the common cube box of all nodes
  (a = per-axis minimum, ext = largest per-axis extent, scale = 2**21/ext),
  q_d = min(floor((c_d - a_d) * scale), 2**21 - 1), bits interleaved with x
  as the most significant of each triple; ties in the sort are broken by the
  original index (a stable sort).
* Cluster tree (Sec. 2.3, (C1)-(C4) and CBC): the node [lo, hi) is split at
  mid = lo + (hi - lo) // 2 into [lo, mid) and [mid, hi) iff hi - lo > C_leaf.
* Bounding boxes Q_tau (Sec. 2.3): per-axis min and max of the nodes.
* Admissibility (Sec. 2.3, eq. admissibilityCondition):
  min(diam Q_tau, diam Q_sigma) <= eta * dist(Q_tau, Q_sigma), with diam the
  Euclidean box diagonal and dist the Euclidean gap between the boxes,
  compared squared in FP64 with the fixed evaluation order
  (a*a + b*b) + c*c and without fused multiply-adds; equality is admissible.
* Block cluster tree (Sec. 2.3, Algorithm 1): a block is subdivided into the
  four products of the children iff it is not admissible and both clusters
  are larger than C_leaf; otherwise it is a leaf.  Children are visited as
  (tau1,sigma1), (tau1,sigma2), (tau2,sigma1), (tau2,sigma2).

All positions below are positions in the Morton-sorted order.
"""
from __future__ import annotations

import numpy as np

MORTON_BITS = 21


def morton_box(C: np.ndarray):
    """(a[3], scale) of the common quantisation cube."""
    a = C.min(axis=0)
    b = C.max(axis=0)
    ext = float(np.max(b - a))
    scale = (2.0 ** MORTON_BITS) / ext if ext > 0.0 else 0.0
    return a, scale


def morton_keys(C: np.ndarray) -> np.ndarray:
    """63-bit Morton keys (uint64) of points C[N, 3]."""
    a, scale = morton_box(C)
    q = np.floor((C - a[None, :]) * scale)
    q = np.minimum(q, float(2 ** MORTON_BITS - 1)).astype(np.uint64)
    key = np.zeros(C.shape[0], dtype=np.uint64)
    for k in range(MORTON_BITS):
        kk = np.uint64(k)
        one = np.uint64(1)
        key |= ((q[:, 0] >> kk) & one) << np.uint64(3 * k + 2)
        key |= ((q[:, 1] >> kk) & one) << np.uint64(3 * k + 1)
        key |= ((q[:, 2] >> kk) & one) << np.uint64(3 * k)
    return key


def morton_order(keys: np.ndarray) -> np.ndarray:
    """pi: Morton position -> original index (ascending key, ties by index)."""
    return np.argsort(keys, kind="stable").astype(np.int64)


def cluster_tree(n: int, leaf_size: int):
    """CBC tree over [0, n) in breadth-first order.

    Returns lo[k], hi[k], child[k] (index of the first child, -1 for a leaf;
    the second child is child[k] + 1) and level[k]."""
    lo, hi, child, level = [0], [n], [], [0]
    k = 0
    while k < len(lo):
        a, b = lo[k], hi[k]
        if b - a > leaf_size:
            mid = a + (b - a) // 2
            child.append(len(lo))
            lo += [a, mid]
            hi += [mid, b]
            level += [level[k] + 1, level[k] + 1]
        else:
            child.append(-1)
        k += 1
    return (np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64),
            np.array(child, dtype=np.int64), np.array(level, dtype=np.int64))


def cluster_boxes(Cs: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """[ncl, 6] boxes (min x,y,z, max x,y,z) of the sorted points Cs."""
    out = np.empty((lo.size, 6))
    for k in range(lo.size):
        p = Cs[lo[k]:hi[k]]
        out[k, :3] = p.min(axis=0)
        out[k, 3:] = p.max(axis=0)
    return out


def diam2(box: np.ndarray) -> np.ndarray:
    """Squared Euclidean diagonal of boxes [..., 6]."""
    dx = box[..., 3] - box[..., 0]
    dy = box[..., 4] - box[..., 1]
    dz = box[..., 5] - box[..., 2]
    return (dx * dx + dy * dy) + dz * dz


def dist2(bt: np.ndarray, bs: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance between boxes bt and bs [..., 6]."""
    g = []
    for d in range(3):
        g1 = bs[..., d] - bt[..., 3 + d]
        g2 = bt[..., d] - bs[..., 3 + d]
        g.append(np.maximum(np.maximum(g1, g2), 0.0))
    return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]


def admissible(bt: np.ndarray, bs: np.ndarray, eta: float) -> np.ndarray:
    """eq. admissibilityCondition in squared form (equality admissible)."""
    return np.minimum(diam2(bt), diam2(bs)) <= (eta * eta) * dist2(bt, bs)


def block_tree_recursive(lo, hi, child, boxes, eta: float, leaf_size: int):
    """Algorithm 1, literally (recursive); for small problems.

    Returns a list of leaves (tau, sigma, admissible)."""
    leaves = []

    def build(t: int, s: int):
        adm = bool(admissible(boxes[t], boxes[s], eta))
        if (not adm) and (hi[t] - lo[t] > leaf_size) and (hi[s] - lo[s] > leaf_size):
            for tc in (child[t], child[t] + 1):
                for sc in (child[s], child[s] + 1):
                    build(tc, sc)
        else:
            leaves.append((t, s, adm))

    build(0, 0)
    return leaves


def block_tree(lo, hi, child, boxes, eta: float, leaf_size: int):
    """Algorithm 1 evaluated breadth-first with arrays (the same recursion,
    visited level by level); used for large problems.

    Returns (tau[], sigma[], admissible[]) of all leaves."""
    t = np.array([0], dtype=np.int64)
    s = np.array([0], dtype=np.int64)
    out_t, out_s, out_a = [], [], []
    while t.size:
        adm = admissible(boxes[t], boxes[s], eta)
        split = (~adm) & (hi[t] - lo[t] > leaf_size) & (hi[s] - lo[s] > leaf_size)
        leaf = ~split
        out_t.append(t[leaf])
        out_s.append(s[leaf])
        out_a.append(adm[leaf])
        ts, ss = t[split], s[split]
        ct, cs = child[ts], child[ss]
        t = np.stack([ct, ct, ct + 1, ct + 1], axis=1).reshape(-1)
        s = np.stack([cs, cs + 1, cs, cs + 1], axis=1).reshape(-1)
    return np.concatenate(out_t), np.concatenate(out_s), np.concatenate(out_a)


class Partition:
    """Everything the clustering stage of the method produces for one mesh."""

    def __init__(self, C: np.ndarray, leaf_size: int, eta: float):
        self.leaf_size = int(leaf_size)
        self.eta = float(eta)
        self.keys = morton_keys(C)
        self.perm = morton_order(self.keys)             # position -> original index
        self.Cs = C[self.perm]
        self.lo, self.hi, self.child, self.level = cluster_tree(C.shape[0], leaf_size)
        self.boxes = cluster_boxes(self.Cs, self.lo, self.hi)
        self.t, self.s, self.adm = block_tree(self.lo, self.hi, self.child, self.boxes,
                                               self.eta, self.leaf_size)

    def leaf_table(self) -> np.ndarray:
        """Rows (row_lo, row_hi, col_lo, col_hi, admissible) sorted
        lexicographically: the canonical form compared for bit-exactness."""
        tab = np.stack([self.lo[self.t], self.hi[self.t], self.lo[self.s], self.hi[self.s],
                        self.adm.astype(np.int64)], axis=1)
        order = np.lexsort(tab.T[::-1])
        return tab[order]
