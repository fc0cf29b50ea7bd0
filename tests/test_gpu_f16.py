"""FP16 factor storage (FP32 evaluation and ACA, FP32 dense blocks, U/V in
FP16 with per-term FP32 scales for U): products against the dense oracle
within exactly 10 eps at the tolerance the form is built for (eps 1e-4), a
separate FP16-vs-FP32 consistency check of the factor rounding, and GMRES to
a 1e-8 residual with respect to the stored operator."""
import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# FP16 keeps 11 significant bits: each stored factor entry is rounded with a
# relative error <= 2^-11 of its column's largest entry; the FP16 and FP32
# forms built on one mesh share ranks and pivots up to float rounding, so
# their products differ by a small multiple of that (consistency only; the
# parity bound against the oracle is 10 eps).
F16_BOUND = 2.0 ** -11
EPS = 1e-4


@pytest.fixture(scope="module")
def small(oracle_ops):
    from synthetic import icosphere
    V, T = icosphere(4)
    op, A = oracle_ops(4, dense=True)
    return V, T, op, A


@pytest.mark.parametrize("nrhs", [1, 5, 16])
def test_f16_products(small, nrhs):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = small
    say("f16 products", nrhs)
    eps = EPS
    H16 = hm.HMatrix(V, T, leaf_size=64, eps=eps, precision="f16")
    H32 = hm.HMatrix(V, T, leaf_size=64, eps=eps, precision="f32")
    assert H16.stats()["precision"] == 2
    assert H16.stats()["stored_bytes"] < H32.stats()["stored_bytes"]
    x = normal_columns(op.n, nrhs, seed=3)
    xt = torch.tensor(x, device=DEV)
    if nrhs == 1:
        xt = xt[:, 0].contiguous()
    for tr in (False, True):
        y16 = H16.matvec(xt, transpose=tr).cpu().numpy().reshape(op.n, -1)
        y32 = H32.matvec(xt, transpose=tr).cpu().numpy().reshape(op.n, -1)
        ref = (A.T if tr else A) @ x
        assert rel2(y32, ref) <= 10 * eps
        assert rel2(y16, ref) <= 10 * eps
        # consistency of the two forms: the FP16 rounding of the factors
        assert rel2(y16, y32) <= 4 * F16_BOUND
    H16.free()
    H32.free()


def test_f16_factors_roundtrip(small):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("f16 factors")
    H = hm.HMatrix(V, T, leaf_size=64, eps=EPS, precision="f16")
    perm = H.perm()
    lb = H.lr_blocks()
    for b in np.random.default_rng(2).choice(len(lb), 20, replace=False):
        r0, r1, c0, c1, rank, _ = lb[b]
        U, Vf = H.lr_factors(int(b))
        assert np.abs(Vf).max() <= 1.0 + 1e-3           # pivot normalisation
        Ab = A[np.ix_(perm[r0:r1], perm[c0:c1])]
        assert np.linalg.norm(Ab - U @ Vf.T) / np.linalg.norm(Ab) <= 10 * EPS
    H.free()


def test_f16_solve_to_1e8(small):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("f16 solve")
    H = hm.HMatrix(V, T, leaf_size=64, eps=1e-4, precision="f16")
    f = torch.ones(op.n, dtype=torch.float64, device=DEV)
    s, info, st = H.solve(f, tol=1e-8, restart=50, max_iter=2000)
    assert st == hm.HM_OK and info.rel_residual <= 1e-8
    # residual with respect to the stored operator, recomputed here
    r = f - H.matvec(s)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(f)) <= 1.5e-8
    s = s.cpu().numpy()
    s_lu = np.linalg.solve(A, np.ones(op.n))
    assert rel2(s, s_lu) <= np.linalg.cond(A) * (10 * EPS + 1e-8)
    H.free()
