"""Writes tests/golden/sphere_errors.json from the oracle only.

The paper prints no values for this collocation discretisation; these are the
oracle's own calibrated values, kept as a regression pin for the oracle."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bem  # noqa: E402
from synthetic import icosphere  # noqa: E402


def main():
    out = {"constant_density_maxerr": {}, "source": "oracle.bem, icosphere levels 2-4, f = 1"}
    for L in (2, 3, 4):
        V, T = icosphere(L)
        op = bem.Operator(V, T)
        A = op.dense()
        out["constant_density_maxerr"][str(L)] = float(np.abs(np.linalg.solve(A, np.ones(op.n)) - 1).max())
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_errors.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
