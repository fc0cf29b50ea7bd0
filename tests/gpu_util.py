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
