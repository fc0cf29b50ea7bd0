"""Closed forms on the unit sphere used to pin the discrete operator.

* A uniform unit density on the unit sphere has single-layer potential 1 on
  the sphere (the shell of charge 4 pi seen from its own surface).
* Spherical harmonics are eigenfunctions: V Y_l = Y_l / (2l + 1).
* The paper's right-hand side f = 4 x1^2 - 3 x2^2 - x3^2 (Sec. 4.3) is a
  harmonic polynomial of degree 2; on the unit sphere its density is 5 f and
  its interior solution is f itself.
"""
from __future__ import annotations

import math

import numpy as np


def legendre(l: int, t: np.ndarray) -> np.ndarray:
    """P_l(t) by the three-term recurrence."""
    p0 = np.ones_like(t)
    if l == 0:
        return p0
    p1 = t.copy()
    for k in range(1, l):
        p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
    return p1


def zonal_harmonic(l: int, x: np.ndarray) -> np.ndarray:
    """Y_l^0(x/|x|) = sqrt((2l+1)/(4 pi)) P_l(z/|x|)."""
    z = x[:, 2] / np.linalg.norm(x, axis=1)
    return math.sqrt((2 * l + 1) / (4.0 * math.pi)) * legendre(l, z)


def paper_rhs(x: np.ndarray) -> np.ndarray:
    """f(x) = 4 x1^2 - 3 x2^2 - x3^2 (Sec. 4.3)."""
    return 4.0 * x[:, 0] ** 2 - 3.0 * x[:, 1] ** 2 - x[:, 2] ** 2
