"""Galerkin discretisation of the single-layer operator -- TEST INFRASTRUCTURE.

Sec. 2.2 (eq. linearSystem) discretises S u = f by Galerkin BEM: with one
piecewise-constant basis function per flat triangle (the paper's trial space
of piecewise constants with nodes at element centres, Sec. 4.1)

    a_ij = int_{T_i} int_{T_j} 1 / (4 pi |x - y|) dsigma_y dsigma_x,
    f_i  = int_{T_i} f dsigma.

(The printed entry formula puts both basis functions at x'; the usual
reading phi_i(x) phi_j(x') is used.)  Sec. 4.1 computes the integrals with
higher-order quadrature and the Duffy trick.  Reading used here:

  * triangles that share no vertex: Radon's seven-point rule on both
    triangles (49 kernel values), the rule that defines the far field of the
    collocation operator too;
  * identical triangles and triangles that share an edge or a vertex: a
    12 x 12 Gauss rule on T_i in collapsed coordinates (outer integral), and
    for every outer point x the inner integral over T_j in closed form.  The
    closed form follows the Duffy / polar decomposition: T_j is split at the
    projection x' of x onto its plane into the three signed triangles
    (x', v_k, v_k+1); in polar coordinates about x' each gives one edge term
    (inner_integral below), so the 1/|x - y| singularity never meets a
    quadrature node.

Everything is FP64, plain NumPy, unblocked.  Only tests, the smoke check and
the benchmark's CPU leg use it.
"""
from __future__ import annotations

import math

import numpy as np

from . import bem, quadrature

FOUR_PI = 4.0 * math.pi
#: Gauss-Legendre points per collapsed coordinate of the outer rule
Q_OUTER = 12


def gauss01(q: int):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def collapsed_rule(a: np.ndarray, b: np.ndarray, c: np.ndarray, q: int):
    """Quadrature on the triangle (a, b, c) in collapsed coordinates with the
    collapsed corner at a: y(s, t) = a + s (b - a) + s t (c - b), s, t in
    [0, 1], dy = s |(b - a) x (c - b)| ds dt.  Returns points [q*q, 3] and
    weights [q*q] (they sum to the area)."""
    g, w = gauss01(q)
    s, t = np.meshgrid(g, g, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    s, t, wgt = s.ravel(), t.ravel(), (ws * wt).ravel()
    pts = a[None, :] + s[:, None] * (b - a)[None, :] + (s * t)[:, None] * (c - b)[None, :]
    jac = np.linalg.norm(np.cross(b - a, c - b))
    return pts, wgt * s * jac


def inner_integral(x: np.ndarray, v0: np.ndarray, v1: np.ndarray, v2: np.ndarray):
    """int_T dsigma_y / |x - y| for the flat triangle T = (v0, v1, v2) and any
    point x (or every row of a [P, 3] array), in closed form.

    With d the signed height of x over the plane of T and x' its projection,
    T is the signed sum of the triangles (x', a, b) over its edges (a, b).
    In polar coordinates (rho, phi) about x', with phi measured from the foot
    point of x' on the edge line (distance h) and l = h tan(phi) the
    coordinate along the edge, the edge is rho = h / cos(phi) and

        int int rho drho dphi / sqrt(rho^2 + d^2)
          = int (sqrt(l^2 + h^2 + d^2) - |d|) dphi,   dphi = h dl / (l^2 + h^2),

    which integrates to h (asinh(l/c)) + |d| atan(|d| l / (h R)) - |d|
    atan(l / h) between the edge's end points (c^2 = h^2 + d^2, R the
    distance from x to the end point).  For d = 0 this is the in-plane formula
    of the collocation self-term."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))     # [P, 3]
    n = np.cross(v1 - v0, v2 - v0)
    nh = n / np.linalg.norm(n)
    d = (x - v0[None, :]) @ nh                             # [P] signed heights
    ad = np.abs(d)
    xp = x - d[:, None] * nh[None, :]
    total = np.zeros(x.shape[0])
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        e = b - a
        le = np.linalg.norm(e)
        t = e / le
        cr = np.cross(a[None, :] - xp, e[None, :]) @ nh    # twice the signed area of (x', a, b)
        h = np.abs(cr) / le
        ok = h > 0.0                                       # x' on the edge line: empty triangle
        hs = np.where(ok, h, 1.0)
        la = (a[None, :] - xp) @ t
        lb = (b[None, :] - xp) @ t
        ra = np.linalg.norm(x - a[None, :], axis=1)
        rb = np.linalg.norm(x - b[None, :], axis=1)
        c = np.sqrt(hs * hs + d * d)
        val = hs * (np.arcsinh(lb / c) - np.arcsinh(la / c)) + _height_terms(ad, hs, la, lb, ra, rb)
        total += np.where(ok, _signed(cr, val), 0.0)
    return total if total.size > 1 else float(total[0])


def _height_terms(ad, h, la, lb, ra, rb):
    """The part of an edge term that a point off the plane adds (zero in the
    plane): |d| (atan(|d| l / (h R)) - atan(l / h)) between the end points."""
    return (ad * (np.arctan(ad * lb / (h * rb)) - np.arctan(ad * la / (h * ra)))
            - ad * (np.arctan(lb / h) - np.arctan(la / h)))


def _signed(cr, val):
    """An edge term with the orientation of its triangle (x', a, b): negative
    when x' lies beyond the edge, so that the three triangles add up to T."""
    return np.where(cr > 0.0, val, -val)


def entry_singular(Ti: np.ndarray, Tj: np.ndarray, q_out: int = Q_OUTER) -> float:
    """a_ij for triangles (3 x 3 vertex arrays) that coincide or touch: outer
    collapsed Gauss rule on T_i, inner integral over T_j in closed form."""
    pts, wgt = collapsed_rule(Ti[0], Ti[1], Ti[2], q_out)
    vals = np.atleast_1d(inner_integral(pts, Tj[0], Tj[1], Tj[2]))
    return float(np.sum(wgt * vals)) / FOUR_PI


def entry_far(Ti: np.ndarray, Tj: np.ndarray) -> float:
    """a_ij with Radon's seven-point rule on both triangles."""
    xi = quadrature.nodes(Ti[0], Ti[1], Ti[2])            # [7, 3]
    yj = quadrature.nodes(Tj[0], Tj[1], Tj[2])
    ai = 0.5 * np.linalg.norm(np.cross(Ti[1] - Ti[0], Ti[2] - Ti[0]))
    aj = 0.5 * np.linalg.norm(np.cross(Tj[1] - Tj[0], Tj[2] - Tj[0]))
    d = np.linalg.norm(xi[:, None, :] - yj[None, :, :], axis=2)
    w = quadrature.WEIGHTS
    return ai * aj * float(np.sum(w[:, None] * w[None, :] / d)) / FOUR_PI


class GalerkinOperator:
    """The dense Galerkin matrix A of a mesh, evaluated on demand."""

    def __init__(self, V: np.ndarray, T: np.ndarray, q_out: int = Q_OUTER):
        self.V = np.asarray(V, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.n = self.T.shape[0]
        self.q_out = q_out
        self.area = bem.areas(self.V, self.T)
        self.y = bem.quad_nodes(self.V, self.T)            # [N, 7, 3]
        # triangles around every vertex: pairs sharing a vertex are singular
        self._around = {}
        for j, tri in enumerate(self.T):
            for v in tri:
                self._around.setdefault(int(v), set()).add(j)

    def touching(self, i: int) -> set:
        """Triangles that share at least one vertex with T_i (T_i included)."""
        out = set()
        for v in self.T[i]:
            out |= self._around[int(v)]
        return out

    def tri(self, i: int) -> np.ndarray:
        return self.V[self.T[i]]

    def block(self, rows, cols) -> np.ndarray:
        """A[rows][:, cols]: the 7 x 7 rule everywhere, then the entries of
        touching pairs replaced by the singular rule."""
        rows = np.asarray(rows, dtype=np.int64).reshape(-1)
        cols = np.asarray(cols, dtype=np.int64).reshape(-1)
        out = np.empty((rows.size, cols.size))
        w = quadrature.WEIGHTS
        yc = self.y[cols]                                   # [c, 7, 3]
        step = max(1, int(2_000_000 // max(cols.size * 49, 1)))
        for s in range(0, rows.size, step):
            r = rows[s:s + step]
            xr = self.y[r]                                  # [r, 7, 3]
            acc = np.zeros((r.size, cols.size))
            with np.errstate(divide="ignore", invalid="ignore"):
                for p in range(7):
                    for q in range(7):
                        d = xr[:, None, p, :] - yc[None, :, q, :]
                        acc += w[p] * w[q] / np.sqrt((d[..., 0] ** 2 + d[..., 1] ** 2) + d[..., 2] ** 2)
            out[s:s + step] = acc * (self.area[r][:, None] * self.area[cols][None, :]) / FOUR_PI
        colpos = {int(c): k for k, c in enumerate(cols)}
        for a, i in enumerate(rows):
            for j in self.touching(int(i)):
                k = colpos.get(j)
                if k is not None:
                    out[a, k] = entry_singular(self.tri(int(i)), self.tri(j), self.q_out)
        return out

    def dense(self) -> np.ndarray:
        return self.block(np.arange(self.n), np.arange(self.n))

    def matvec_rows(self, x: np.ndarray, rows) -> np.ndarray:
        """(A x)[rows] from exact rows."""
        x = np.asarray(x, dtype=np.float64)
        rows = np.asarray(rows, dtype=np.int64)
        out = []
        step = max(1, int(300_000 // max(self.n, 1)))
        for s in range(0, rows.size, step):
            out.append(self.block(rows[s:s + step], np.arange(self.n)) @ x)
        return np.concatenate(out) if out else np.zeros((0,) + x.shape[1:])

    def rhs(self, f) -> np.ndarray:
        """f_i = int_{T_i} f dsigma with the seven-point rule; f maps
        points [..., 3] to values [...]."""
        return self.area * np.sum(quadrature.WEIGHTS[None, :] * f(self.y), axis=1)


def potential(V: np.ndarray, T: np.ndarray, sigma: np.ndarray, points: np.ndarray) -> np.ndarray:
    """The single-layer potential of the piecewise-constant density sigma at
    points away from the surface (Sec. 2.1, eq. singleLayerPotential), with
    the seven-point rule on every triangle."""
    return bem.Operator(V, T).potential(sigma, points)
