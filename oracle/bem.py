"""Laplace single-layer operator, collocation with piecewise constants.

Sec. 2.1 (Example 1, eqs. singleLayerPotential and
exampleBoundaryIntegralEquation) defines S u (x) = int_Gamma u(y) / (4 pi
|x - y|) dsigma_y = f(x) on the surface.  The paper discretises it by
Galerkin BEM (Sec. 2.2); here it is collocation, the alternative named
in Sec. 1, with nodes at element centres as in Sec. 4.1: one unknown per flat
triangle T_j, collocation point x_i = centroid of T_i, and

    a_ij = int_{T_j} G(x_i, y) dsigma_y,     G(x, y) = 1 / (4 pi |x - y|),

evaluated with the seven-point rule for i != j and in closed form for i == j
(x_i lies in the plane of T_i).  Everything here is FP64 and unblocked.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature

FOUR_PI = 4.0 * math.pi


def _verts(V: np.ndarray, T: np.ndarray):
    return V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]


def centroids(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Collocation points x_i = ((v0 + v1) + v2) / 3, rounded at every step
    (the bit-exact clustering depends on these values)."""
    v0, v1, v2 = _verts(V, T)
    return ((v0 + v1) + v2) / 3.0


def areas(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """|T_j| = |(v1 - v0) x (v2 - v0)| / 2."""
    v0, v1, v2 = _verts(V, T)
    return 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0), axis=1)


def quad_nodes(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """[N, 7, 3] quadrature nodes of every triangle."""
    v0, v1, v2 = _verts(V, T)
    return quadrature.nodes(v0, v1, v2)


def self_integral(x: np.ndarray, v0: np.ndarray, v1: np.ndarray, v2: np.ndarray) -> np.ndarray:
    """int_T dsigma_y / |x - y| for x inside the (flat) triangle T = (v0,v1,v2).

    Split T at x into the three triangles (x, v_a, v_b) over its edges.  In
    polar coordinates about x, with the angle measured from the foot of the
    perpendicular onto the edge line (distance h), the edge is r = h/cos(phi)
    and the integrand r * (1/r) leaves int h/cos(phi) dphi = h ln(sec + tan).
    With sec = R/h and tan = l/h (R the distance to an edge end point, l its
    signed coordinate along the edge measured from the foot point) each edge
    contributes h * ln((R_b + l_b) / (R_a + l_a)).
    """
    total = np.zeros(x.shape[0])
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        e = b - a
        le = np.linalg.norm(e, axis=1)
        t = e / le[:, None]
        la = np.einsum("ij,ij->i", a - x, t)          # signed coordinate of a
        lb = np.einsum("ij,ij->i", b - x, t)          # signed coordinate of b
        foot = a - la[:, None] * t                    # foot point of x on the edge line
        h = np.linalg.norm(foot - x, axis=1)
        ra = np.linalg.norm(a - x, axis=1)
        rb = np.linalg.norm(b - x, axis=1)
        total += h * np.log((rb + lb) / (ra + la))
    return total


def self_terms(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Diagonal entries a_ii = (1/4pi) int_{T_i} dsigma_y / |x_i - y|."""
    v0, v1, v2 = _verts(V, T)
    return self_integral(centroids(V, T), v0, v1, v2) / FOUR_PI


class Operator:
    """The dense collocation matrix A of a mesh, evaluated on demand."""

    def __init__(self, V: np.ndarray, T: np.ndarray):
        self.V = np.asarray(V, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.n = self.T.shape[0]
        self.x = centroids(self.V, self.T)
        self.area = areas(self.V, self.T)
        self.y = quad_nodes(self.V, self.T)
        self.diag = self_terms(self.V, self.T)

    # -- entries -----------------------------------------------------------
    def block(self, rows, cols) -> np.ndarray:
        """A[rows][:, cols] for index arrays rows, cols (any order)."""
        rows = np.asarray(rows, dtype=np.int64).reshape(-1)
        cols = np.asarray(cols, dtype=np.int64).reshape(-1)
        out = np.empty((rows.size, cols.size))
        step = max(1, int(4_000_000 // max(cols.size, 1)))
        y = self.y[cols]                                   # [c, 7, 3]
        wa = self.area[cols] / FOUR_PI                     # [c]
        for s in range(0, rows.size, step):
            r = rows[s:s + step]
            xr = self.x[r]
            acc = np.zeros((r.size, cols.size))
            with np.errstate(divide="ignore", invalid="ignore"):
                for q in range(quadrature.WEIGHTS.size):
                    d0 = xr[:, 0, None] - y[None, :, q, 0]
                    d1 = xr[:, 1, None] - y[None, :, q, 1]
                    d2 = xr[:, 2, None] - y[None, :, q, 2]
                    acc += quadrature.WEIGHTS[q] / np.sqrt((d0 * d0 + d1 * d1) + d2 * d2)
            vals = acc * wa[None, :]
            same = r[:, None] == cols[None, :]
            if same.any():
                vals = np.where(same, self.diag[cols][None, :], vals)
            out[s:s + step] = vals
        return out

    def rows(self, rows) -> np.ndarray:
        """Exact rows A[rows, :]."""
        return self.block(rows, np.arange(self.n))

    def cols(self, cols) -> np.ndarray:
        """Exact columns A[:, cols]."""
        return self.block(np.arange(self.n), cols)

    def dense(self) -> np.ndarray:
        """The full N x N matrix (small N only)."""
        return self.block(np.arange(self.n), np.arange(self.n))

    def matvec_rows(self, x: np.ndarray, rows) -> np.ndarray:
        """(A x)[rows] computed directly from exact rows."""
        x = np.asarray(x, dtype=np.float64)
        rows = np.asarray(rows, dtype=np.int64)
        out = []
        step = max(1, int(2_000_000 // max(self.n, 1)))
        for s in range(0, rows.size, step):
            out.append(self.rows(rows[s:s + step]) @ x)
        return np.concatenate(out) if out else np.zeros((0,) + x.shape[1:])

    def rmatvec_cols(self, x: np.ndarray, cols) -> np.ndarray:
        """(A^T x)[cols] computed directly from exact columns."""
        x = np.asarray(x, dtype=np.float64)
        cols = np.asarray(cols, dtype=np.int64)
        out = []
        step = max(1, int(2_000_000 // max(self.n, 1)))
        for s in range(0, cols.size, step):
            out.append(self.cols(cols[s:s + step]).T @ x)
        return np.concatenate(out) if out else np.zeros((0,) + x.shape[1:])

    # -- single-layer potential off the surface (Sec. 2.1, eq. singleLayerPotential)
    def potential(self, sigma: np.ndarray, points: np.ndarray) -> np.ndarray:
        """U(p) = sum_j sigma_j int_{T_j} G(p, y) dsigma_y with the 7-point rule,
        for points p away from the surface (the paper's interior error test,
        Sec. 4.3)."""
        points = np.asarray(points, dtype=np.float64)
        out = np.empty(points.shape[0])
        wa = self.area / FOUR_PI
        step = max(1, int(4_000_000 // max(self.n * 7, 1)))
        for s in range(0, points.shape[0], step):
            d = points[s:s + step][:, None, None, :] - self.y[None]
            dist = np.sqrt(((d[..., 0] ** 2 + d[..., 1] ** 2) + d[..., 2] ** 2))
            g = (quadrature.WEIGHTS[None, None, :] / dist).sum(-1) * wa[None, :]
            out[s:s + step] = g @ sigma
        return out


def solve_dense(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    """sigma = A^{-1} f by LU (numpy.linalg.solve); the textbook reference
    for the iterative solve on small problems."""
    return np.linalg.solve(A, f)
