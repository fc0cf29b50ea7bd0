"""Adaptive cross approximation with partial pivoting (Sec. 2.3).

The paper describes ACA as a pivoted Gauss elimination that builds the
low-rank factors U V^T of an admissible block by successive rank-one
updates, from O(k (m + n)) entries of the block.  It fixes neither the
pivoting nor the stopping rule; this oracle follows the partially pivoted
variant (Bebendorf 2000) with these readings:

* the first pivot row is row 0 of the block (local Morton order);
* step r: residual row  v~ = a(i*, :) - sum_l u_l[i*] v_l;  pivot column
  j* = argmax |v~| (ties: smallest index); delta = v~[j*];
  v_r = v~ / delta;  residual column u_r = a(:, j*) - sum_l v_l[j*] u_l;
* a zero pivot (delta == 0) marks the row as reproduced and moves to the
  unused row with the largest |u_{r-1}| (smallest unused row if r == 0);
* ||S_r||_F^2 = ||S_{r-1}||_F^2 + 2 sum_{l<r} (u_l.u_r)(v_l.v_r)
  + ||u_r||^2 ||v_r||^2, and the method stops after keeping term r when
  ||u_r|| ||v_r|| <= eps ||S_r||_F, or when r reaches kmax or min(m, n),
  or when every row has been used;
* the next pivot row is the unused row with the largest |u_r| (ties:
  smallest index).
"""
from __future__ import annotations

import math

import numpy as np


def aca(row, col, m: int, n: int, eps: float, kmax: int):
    """Cross approximation of an m x n block given entry accessors
    row(i) -> a(i, :) and col(j) -> a(:, j).  Returns U [m, r], V [n, r]."""
    kmax = min(int(kmax), m, n)
    us, vs = [], []
    used = np.zeros(m, dtype=bool)
    i_star = 0
    s2 = 0.0
    while True:
        v_t = np.array(row(i_star), dtype=np.float64)
        for u_l, v_l in zip(us, vs):
            v_t -= u_l[i_star] * v_l
        used[i_star] = True
        j_star = int(np.argmax(np.abs(v_t)))
        delta = v_t[j_star]
        if delta == 0.0:
            if used.all():
                break
            free = np.flatnonzero(~used)
            if us:
                i_star = int(free[np.argmax(np.abs(us[-1][free]))])
            else:
                i_star = int(free[0])
            continue
        v = v_t / delta
        u = np.array(col(j_star), dtype=np.float64)
        for u_l, v_l in zip(us, vs):
            u -= v_l[j_star] * u_l
        cross = 0.0
        for u_l, v_l in zip(us, vs):
            cross += float(u_l @ u) * float(v_l @ v)
        uu = float(u @ u)
        vv = float(v @ v)
        s2 += 2.0 * cross + uu * vv
        us.append(u)
        vs.append(v)
        if math.sqrt(uu) * math.sqrt(vv) <= eps * math.sqrt(max(s2, 0.0)):
            break
        if len(us) >= kmax or used.all():
            break
        free = np.flatnonzero(~used)
        i_star = int(free[np.argmax(np.abs(u[free]))])
    U = np.stack(us, axis=1) if us else np.zeros((m, 0))
    V = np.stack(vs, axis=1) if vs else np.zeros((n, 0))
    return U, V


def aca_dense(A: np.ndarray, eps: float, kmax: int | None = None):
    """ACA of an explicitly given block."""
    m, n = A.shape
    return aca(lambda i: A[i, :], lambda j: A[:, j], m, n, eps,
               min(m, n) if kmax is None else kmax)
