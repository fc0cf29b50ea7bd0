"""Radon's seven-point, degree-5 quadrature rule on a triangle (Stroud T2:5-1).

The off-diagonal collocation entries integrate the single-layer kernel of
Sec. 2.1 (eq. singleLayerPotential) over a flat source triangle with this
rule.  Nodes are given in barycentric coordinates; the weights sum to one and
are multiplied by the triangle's area.
"""
from __future__ import annotations

import math

import numpy as np

_S15 = math.sqrt(15.0)
_A1 = (6.0 - _S15) / 21.0
_B1 = (9.0 + 2.0 * _S15) / 21.0
_A2 = (6.0 + _S15) / 21.0
_B2 = (9.0 - 2.0 * _S15) / 21.0
_W0 = 9.0 / 40.0
_W1 = (155.0 - _S15) / 1200.0
_W2 = (155.0 + _S15) / 1200.0

#: barycentric coordinates (lambda0, lambda1, lambda2) of the 7 nodes
BARY = np.array([
    [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
    [_A1, _A1, _B1], [_A1, _B1, _A1], [_B1, _A1, _A1],
    [_A2, _A2, _B2], [_A2, _B2, _A2], [_B2, _A2, _A2],
], dtype=np.float64)

#: weights, normalised so that they sum to 1 (multiply by the area)
WEIGHTS = np.array([_W0, _W1, _W1, _W1, _W2, _W2, _W2], dtype=np.float64)


def nodes(v0: np.ndarray, v1: np.ndarray, v2: np.ndarray) -> np.ndarray:
    """Quadrature nodes y_q = l0*v0 + l1*v1 + l2*v2 for triangles given by
    vertex arrays [..., 3]; returns [..., 7, 3]."""
    l0 = BARY[:, 0][:, None]
    l1 = BARY[:, 1][:, None]
    l2 = BARY[:, 2][:, None]
    return (l0 * v0[..., None, :] + l1 * v1[..., None, :]) + l2 * v2[..., None, :]
