"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def leaf_table_from_gpu(H):
    """Canonical sorted (row_lo, row_hi, col_lo, col_hi, adm) table of the
    library's partition."""
    d = H.dense_blocks()[:, :4]
    a = H.lr_blocks()[:, :4]
    tab = np.concatenate([np.c_[d, np.zeros(len(d), dtype=np.int64)],
                          np.c_[a, np.ones(len(a), dtype=np.int64)]])
    return tab[np.lexsort(tab.T[::-1])]


def rel2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


#: unit roundoff of FP64
U64 = 2.0 ** -53


def node_rounding_tol(op, rows, cols, floor=1e-14):
    """Element-wise relative tolerance of FP64 collocation entries a(i, j),
    i != j, set by the rounding of the quadrature nodes.  Any formula for
    the nodes of the seven-point rule (barycentric sums of the vertices, or
    the centroid plus a multiple of a vertex offset) places each node
    coordinate within about 2u R of its exact value (u the unit roundoff, R
    the largest vertex coordinate), so each distance |x_i - y_jq| carries an
    absolute error of at most 2 sqrt(3) u R and the weighted sum of the
    reciprocal distances a relative error of at most that over the smallest
    distance d_min(i, j).  Two such evaluations differ by at most twice
    that: 8 u R / d_min, and at least `floor`.  Distances are the oracle's
    own node positions; diagonal entries (self-terms) keep `floor`."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    R = float(np.abs(op.V).max())
    d = np.linalg.norm(op.x[rows][..., None, :] - op.y[cols], axis=-1).min(axis=-1)
    tol = np.maximum(floor, 8.0 * U64 * R / np.where(d > 0, d, np.inf))
    return np.where(rows == cols, floor, tol)
