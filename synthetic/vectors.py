"""Seeded random vectors (PCG64 via numpy.random.default_rng)."""
from __future__ import annotations

import numpy as np


def normal_columns(n: int, ncols: int, seed: int = 0) -> np.ndarray:
    """[n, ncols] FP64 N(0,1) matrix from default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((n, ncols))


def sample_rows(n: int, count: int, seed: int = 1) -> np.ndarray:
    """`count` distinct row indices in [0, n), drawn without replacement from
    default_rng(seed), returned sorted."""
    count = min(count, n)
    return np.sort(np.random.default_rng(seed).choice(n, count, replace=False))
