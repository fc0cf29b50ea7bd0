"""Synthetic surface meshes standing in for the paper's geometries.

The paper measures on a parametric cube mesh and a gearwheel mesh that are
not available; smooth icospheres (and radially perturbed spheres) of the
same unknown counts stand in for them.  An icosphere refined L times has
N = 20 * 4**L flat triangles; every unknown is one triangle.

All arithmetic is FP64.  Triangles are oriented with outward normals.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

_PHI = (1.0 + math.sqrt(5.0)) / 2.0


def _icosahedron():
    v = np.array([
        [-1.0, _PHI, 0.0], [1.0, _PHI, 0.0], [-1.0, -_PHI, 0.0], [1.0, -_PHI, 0.0],
        [0.0, -1.0, _PHI], [0.0, 1.0, _PHI], [0.0, -1.0, -_PHI], [0.0, 1.0, -_PHI],
        [_PHI, 0.0, -1.0], [_PHI, 0.0, 1.0], [-_PHI, 0.0, -1.0], [-_PHI, 0.0, 1.0],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return v, t


def _refine(v: np.ndarray, t: np.ndarray):
    """Split every triangle (a,b,c) into four; midpoints are shared per edge
    and projected back to the unit sphere."""
    nv = v.shape[0]
    a, b, c = t[:, 0].astype(np.int64), t[:, 1].astype(np.int64), t[:, 2].astype(np.int64)
    edges = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)])
    key = np.minimum(edges[:, 0], edges[:, 1]) * nv + np.maximum(edges[:, 0], edges[:, 1])
    ukey, inv = np.unique(key, return_inverse=True)
    e0 = ukey // nv
    e1 = ukey % nv
    mid = (v[e0] + v[e1]) * 0.5
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    m = inv.reshape(3, -1) + nv          # m[0]=ab, m[1]=bc, m[2]=ca
    mab, mbc, mca = m[0], m[1], m[2]
    nt = np.concatenate([
        np.stack([a, mab, mca], 1),
        np.stack([mab, b, mbc], 1),
        np.stack([mca, mbc, c], 1),
        np.stack([mab, mbc, mca], 1),
    ]).astype(np.int32)
    return np.concatenate([v, mid]), nt


def icosphere(level: int):
    """Unit icosphere refined `level` times: returns (V[nv,3] f64, T[N,3] i32),
    N = 20*4**level.  Triangle order is deterministic (four children blocks
    appended per refinement), which is *not* a spatial order: the method's
    own Morton sort has to find the locality."""
    if level < 0:
        raise ValueError("level must be >= 0")
    v, t = _icosahedron()
    for _ in range(level):
        v, t = _refine(v, t)
    return np.ascontiguousarray(v), np.ascontiguousarray(t)


def _real_sph_harm(l: int, m: int, xyz: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_lm at unit vectors xyz (via the
    associated Legendre functions from scipy)."""
    from scipy.special import sph_harm_y  # type: ignore
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    ym = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * ym.real
    if m < 0:
        return math.sqrt(2.0) * (-1) ** m * ym.imag
    return ym.real


def perturbed_sphere(level: int, seed: int, amplitude: float = 0.1, lmax: int = 4):
    """Icosphere whose vertices are moved radially to
    r(x) = 1 + amplitude * sum_{l=1..lmax} sum_m c_lm Y_lm(x),  c_lm = z/l**2,
    z ~ N(0,1) drawn in (l, m=-l..l) order from default_rng(seed).
    Degree 0 is skipped (it only rescales the sphere)."""
    v, t = icosphere(level)
    rng = np.random.default_rng(seed)
    r = np.ones(v.shape[0])
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            c = rng.standard_normal() / (l * l)
            r += amplitude * c * _real_sph_harm(l, m, v)
    if r.min() <= 0.5:
        raise ValueError(f"seed {seed}: radial perturbation too large (min r={r.min():.3f})")
    return np.ascontiguousarray(v * r[:, None]), t


def with_near_duplicates(v: np.ndarray, t: np.ndarray, count: int, shift: float, seed: int):
    """The mesh (v, t) plus `count` extra triangles, each a copy of a randomly
    chosen triangle (default_rng(seed)) moved by `shift` along one of its
    edges: distinct triangles whose centres lie within `shift` of each
    other, so that their Morton keys can tie.  The copies are appended after
    the original triangles, with their own vertices."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(t.shape[0], count, replace=False)
    tri = v[t[pick]]                                   # [count, 3, 3]
    e = tri[:, 1] - tri[:, 0]
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    moved = tri + shift * e[:, None, :]
    nv = v.shape[0]
    v2 = np.concatenate([v, moved.reshape(-1, 3)])
    t2 = np.concatenate([t, (nv + np.arange(3 * count)).reshape(count, 3)]).astype(np.int32)
    return np.ascontiguousarray(v2), np.ascontiguousarray(t2)


def mesh_sha256(v: np.ndarray, t: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(v, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(t, dtype=np.int32).tobytes())
    return h.hexdigest()
