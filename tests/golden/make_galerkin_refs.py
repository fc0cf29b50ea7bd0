"""Writes tests/golden/galerkin_icosphere_L8_refs.npz from the oracle only.

Exact rows of A X and of A^T X for the Galerkin matrix with piecewise
constants (Sec. 2.2, eq. linearSystem; oracle/galerkin.py) of the unit
icosphere refined 8 times, N = 1,310,720; X = four N(0,1) columns from
default_rng(0); 256 indices drawn without replacement from default_rng(1).
A column of A is evaluated as a block of all rows by one column, so the
transposed values come from the operator's own entries, not from its
approximate symmetry.  About 1,000 CPU-seconds, so the values are stored.

Run:  python tests/golden/make_galerkin_refs.py [workers]
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import galerkin  # noqa: E402
from synthetic import icosphere, mesh_sha256, normal_columns, sample_rows  # noqa: E402

LEVEL, NCOL, NROW = 8, 4, 256
_OP = None
_X = None


def _rows(idx):
    return _OP.matvec_rows(_X, idx)


def _cols(idx):
    # (A^T X)[c] = sum_i A[i, c] X[i]: column c of A against X
    out = np.empty((len(idx), _X.shape[1]))
    allrows = np.arange(_OP.n)
    for k, c in enumerate(idx):
        out[k] = _OP.block(allrows, [int(c)])[:, 0] @ _X
    return out


def main():
    global _OP, _X
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else len(os.sched_getaffinity(0))
    V, T = icosphere(LEVEL)
    n = T.shape[0]
    _OP = galerkin.GalerkinOperator(V, T)
    _X = normal_columns(n, NCOL, seed=0)
    rows = sample_rows(n, NROW, seed=1)
    chunks = [rows[i::workers] for i in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        yr = pool.map(_rows, chunks)
        yc = pool.map(_cols, chunks)
    y = np.empty((NROW, NCOL))
    yT = np.empty((NROW, NCOL))
    for i in range(workers):
        y[i::workers] = yr[i]
        yT[i::workers] = yc[i]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "galerkin_icosphere_L8_refs.npz")
    np.savez(path, level=LEVEL, n=n, rows=rows, y=y, yT=yT, x_seed=0, row_seed=1,
             mesh_sha256=mesh_sha256(V, T))
    print(f"wrote {path}: {NROW} rows and columns, {NCOL} right-hand sides, "
          f"{time.perf_counter() - t0:.0f} s on {workers} processes")


if __name__ == "__main__":
    main()
