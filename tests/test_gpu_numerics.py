"""Numerical parity of entries, ACA blocks, products and solves (GPU vs the
CPU FP64 oracle)."""
import numpy as np
import pytest
import torch

from gpu_util import node_rounding_tol, rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def small(oracle_ops):
    from synthetic import icosphere
    V, T = icosphere(3)
    op, A = oracle_ops(3, dense=True)
    return V, T, op, A


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 2e-6)])
def test_entries(small, prec, tol):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("entries", prec)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, op.n, 4000)
    cols = rng.integers(0, op.n, 4000)
    rows[:50] = cols[:50]                           # diagonal (self-terms)
    nb = np.argsort(np.linalg.norm(op.x[rows[50:100]][:, None] - op.x[None], axis=-1), axis=1)[:, 1]
    cols[50:100] = nb                               # nearest neighbours (adjacent panels)
    got = H.entries(rows, cols)
    ref = A[rows, cols]
    if prec == "f64":
        tol = node_rounding_tol(op, rows, cols, floor=tol)
    assert np.all(np.abs(got - ref) / np.abs(ref) <= tol)
    H.free()


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_aca_blocks_vs_exact(small, eps):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("aca blocks eps", eps)
    H = hm.HMatrix(V, T, leaf_size=32, eps=eps, precision="f64")
    perm = H.perm()
    lb = H.lr_blocks()
    rng = np.random.default_rng(1)
    for b in rng.choice(len(lb), min(60, len(lb)), replace=False):
        r0, r1, c0, c1, rank, cap = lb[b]
        U, Vf = H.lr_factors(int(b))
        Ab = A[np.ix_(perm[r0:r1], perm[c0:c1])]
        err = np.linalg.norm(Ab - U @ Vf.T) / np.linalg.norm(Ab)
        assert err <= 10 * eps, (b, rank, err)
    H.free()


@pytest.mark.parametrize("prec,eps,bound", [("f64", 1e-6, 1e-5), ("f64", 1e-8, 1e-7),
                                            ("f32", 1e-5, 1e-4)])
@pytest.mark.parametrize("nrhs", [1, 3, 12, 16, 19])
def test_matvec_small_dense(small, prec, eps, bound, nrhs):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = small
    say("matvec", prec, eps, nrhs)
    H = hm.HMatrix(V, T, leaf_size=32, eps=eps, precision=prec)
    x = normal_columns(op.n, nrhs, seed=0)
    for vdt in (torch.float64, torch.float32):
        xt = torch.tensor(x, dtype=vdt, device=DEV)
        if nrhs == 1:
            xt = xt[:, 0].contiguous()
        y = H.matvec(xt).double().cpu().numpy().reshape(op.n, -1)
        yT = H.matvec_T(xt).double().cpu().numpy().reshape(op.n, -1)
        b = bound if vdt == torch.float64 else max(bound, 1e-6)
        ref, refT = A @ x, A.T @ x
        for k in range(nrhs):                     # every column on its own
            assert rel2(y[:, k], ref[:, k]) <= b
            assert rel2(yT[:, k], refT[:, k]) <= b
    H.free()


def test_matvec_deterministic(small):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = small
    say("determinism")
    x = torch.tensor(normal_columns(op.n, 4, seed=2), device=DEV)
    outs = []
    for _ in range(2):
        H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision="f32")
        outs.append((H.matvec(x).cpu().numpy(), H.matvec(x).cpu().numpy(),
                     H.matvec_T(x).cpu().numpy()))
        H.free()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[0][0], outs[0][1])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_solve_constant_density(small, prec):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("solve", prec)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec)
    f = torch.ones(op.n, dtype=torch.float64, device=DEV)
    s, info, st = H.solve(f, tol=1e-10, restart=100, max_iter=500)
    assert st == hm.HM_OK and info.converged == 1
    s = s.cpu().numpy()
    s_lu = np.linalg.solve(A, np.ones(op.n))
    kappa = np.linalg.cond(A)
    # H differs from A by at most ~10 eps; the solution error follows kappa
    assert rel2(s, s_lu) <= kappa * 20 * 1e-6
    res = np.linalg.norm(A @ s - 1) / np.sqrt(op.n)
    assert res <= 1e-10 + 20 * 1e-6 * np.linalg.norm(A, 2) * np.linalg.norm(s) / np.sqrt(op.n)
    # the H-matrix solve inherits the discretisation: sigma ~ 1
    assert np.abs(s - 1).max() < 2e-2
    H.free()


def test_solve_transposed_and_multi_rhs(small):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = small
    say("solve transposed multi rhs")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-8, precision="f64")
    F = normal_columns(op.n, 3, seed=5)
    f = torch.tensor(F, device=DEV)
    s, info, st = H.solve(f, tol=1e-9, restart=30, max_iter=600, transpose=True)
    assert st == hm.HM_OK and info.converged == 3 and info.restarts >= 1
    S = s.cpu().numpy()
    ref = np.linalg.solve(A.T, F)
    assert rel2(S, ref) <= np.linalg.cond(A) * 1e-7


def test_solve_not_converged_status(small):
    import paper_1806_11558_amd as hm
    V, T, op, A = small
    say("solve not converged")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision="f64")
    f = torch.ones(op.n, dtype=torch.float64, device=DEV)
    s, info, st = H.solve(f, tol=1e-14, restart=5, max_iter=3)
    assert st == hm.HM_NOT_CONVERGED and info.iters == 3 and info.converged == 0


@pytest.mark.parametrize("level,nsub,leaf", [(0, 1, 32), (1, 2, 32), (2, 33, 32), (3, 777, 13)])
def test_edge_sizes(level, nsub, leaf):
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere, normal_columns
    V, T = icosphere(level)
    T = T[:nsub]
    say("edge sizes", nsub, leaf)
    op = bem.Operator(V, T)
    A = op.dense()
    H = hm.HMatrix(V, T, leaf_size=leaf, eps=1e-8, precision="f64")
    x = normal_columns(op.n, 2, seed=4)
    y = H.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    yT = H.matvec_T(torch.tensor(x, device=DEV)).cpu().numpy()
    assert rel2(y, A @ x) <= 1e-7 and rel2(yT, A.T @ x) <= 1e-7
    H.free()


@pytest.mark.parametrize("prec,eps", [("f64", 1e-8), ("f32", 1e-6)])
def test_lr_factors_odd_sizes(prec, eps):
    """Stored factors of blocks with odd row and column counts (777
    triangles, leaf 13), read back through HM_Q_LR_FACTORS, against the
    exact blocks within 10 eps; blocks of every rank parity, rank 0
    included when one occurs."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere
    V, T = icosphere(3)
    T = T[:777]
    op = bem.Operator(V, T)
    A = op.dense()
    H = hm.HMatrix(V, T, leaf_size=13, eps=eps, precision=prec)
    perm = H.perm()
    lb = H.lr_blocks()
    odd = np.nonzero(((lb[:, 1] - lb[:, 0]) + (lb[:, 3] - lb[:, 2])) % 2 == 1)[0]
    say("lr factors odd sizes", prec, len(odd), "of", len(lb))
    assert len(odd) > 0
    for b in odd[:40].tolist():
        r0, r1, c0, c1, rank, cap = lb[b]
        U, Vf = H.lr_factors(int(b))
        assert U.shape == (r1 - r0, rank) and Vf.shape == (c1 - c0, rank)
        Ab = A[np.ix_(perm[r0:r1], perm[c0:c1])]
        err = np.linalg.norm(Ab - U @ Vf.T) / np.linalg.norm(Ab)
        assert err <= 10 * eps, (b, rank, err)
    H.free()


@pytest.mark.parametrize("nsub,leaf,ld", [(1000, 8, 8), (1000, 32, 32), (1280, 64, 40),
                                           (1000, 64, 64)])
@pytest.mark.parametrize("prec,eps,bound", [("f64", 1e-8, 1e-7), ("f32", 1e-6, 1e-5)])
def test_products_every_row_tile_count(nsub, leaf, ld, prec, eps, bound):
    """Leaves padded to ld = 8, 32, 40 and 64 rows: the 16-row tiles of the
    MFMA products (1..4), the pass counts of phase 1 and the granule rows of
    the one-column kernels all occur.  Forward and transposed products with
    1, 8 and 16 right-hand sides, double vectors (and float vectors for the
    FP32 form: the single-precision MFMA passes), every column against the
    dense oracle."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere, normal_columns
    V, T = icosphere(3)
    T = T[:nsub]
    say("tile counts", nsub, leaf, prec)
    op = bem.Operator(V, T)
    A = op.dense()
    H = hm.HMatrix(V, T, leaf_size=leaf, eps=eps, precision=prec)
    lv = H.leaves()                               # (lo, size, ld) per leaf
    assert int(lv[:, 2].max()) == ld
    vdts = (torch.float64, torch.float32) if prec == "f32" else (torch.float64,)
    for nrhs in (1, 8, 16):
        x = normal_columns(op.n, nrhs, seed=nrhs)
        ref, refT = A @ x, A.T @ x
        for vdt in vdts:
            xt = torch.tensor(x[:, 0] if nrhs == 1 else x, dtype=vdt, device=DEV)
            y = H.matvec(xt).double().cpu().numpy().reshape(op.n, -1)
            yT = H.matvec_T(xt).double().cpu().numpy().reshape(op.n, -1)
            for k in range(nrhs):
                assert rel2(y[:, k], ref[:, k]) <= bound, (nrhs, k, vdt)
                assert rel2(yT[:, k], refT[:, k]) <= bound, (nrhs, k, vdt)
    H.free()


@pytest.mark.parametrize("prec,eps,bound", [("f64", 1e-8, 1e-7), ("f32", 1e-6, 1e-5)])
def test_products_31_columns(prec, eps, bound):
    """31 right-hand sides in one call run as passes of 16, 8, 4, 2 and 1
    columns (every pass width of the forward and transposed kernels, in
    FP64 with the MFMA passes); every column against the dense oracle at
    N = 1,280."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere, normal_columns
    V, T = icosphere(3)
    say("31 columns", prec)
    op = bem.Operator(V, T)
    A = op.dense()
    H = hm.HMatrix(V, T, leaf_size=32, eps=eps, precision=prec)
    x = normal_columns(op.n, 31, seed=31)
    ref, refT = A @ x, A.T @ x
    for vdt in ((torch.float64, torch.float32) if prec == "f32" else (torch.float64,)):
        xt = torch.tensor(x, dtype=vdt, device=DEV)
        y = H.matvec(xt).double().cpu().numpy()
        yT = H.matvec_T(xt).double().cpu().numpy()
        for k in range(31):
            assert rel2(y[:, k], ref[:, k]) <= bound, (k, vdt)
            assert rel2(yT[:, k], refT[:, k]) <= bound, (k, vdt)
    H.free()


def test_products_ranks_above_64():
    """Leaf 8, eta 5, ACA eps 1e-14, max_rank 128 at N = 1,280: the largest
    admissible blocks (80 x 80) reach ranks above 64, so phase 1 and the
    transposed block sums take their terms 64 at a time.  Forward and
    transposed products with 1, 2, 4, 8 and 16 right-hand sides against the
    dense oracle."""
    import paper_1806_11558_amd as hm
    from oracle import bem
    from synthetic import icosphere, normal_columns
    V, T = icosphere(3)
    say("ranks above 64")
    op = bem.Operator(V, T)
    A = op.dense()
    H = hm.HMatrix(V, T, leaf_size=8, eta=5.0, eps=1e-14, max_rank=128, precision="f64")
    assert H.stats()["rank_max"] > 64
    for nrhs in (1, 2, 4, 8, 16):
        x = normal_columns(op.n, nrhs, seed=20 + nrhs)
        xt = torch.tensor(x[:, 0] if nrhs == 1 else x, device=DEV)
        y = H.matvec(xt).cpu().numpy().reshape(op.n, -1)
        yT = H.matvec_T(xt).cpu().numpy().reshape(op.n, -1)
        ref, refT = A @ x, A.T @ x
        for k in range(nrhs):
            assert rel2(y[:, k], ref[:, k]) <= 1e-10, (nrhs, k)
            assert rel2(yT[:, k], refT[:, k]) <= 1e-10, (nrhs, k)
    H.free()


def test_zonal_harmonic_solves_n81920_fp32():
    """f = Y_l (l = 0..8, nine right-hand sides in one solve) at N = 81,920,
    FP32 form, eps 1e-5, GMRES to 1e-6.  The continuous solution is
    (2l+1) Y_l; the discrete one differs by the discretisation error, which
    must fall under half of the dense oracle's error at N = 5,120 (first order
    in h would give a quarter)."""
    import paper_1806_11558_amd as hm
    from oracle import bem, sphere
    from synthetic import icosphere
    say("zonal harmonics N=81920 f32")
    ls = list(range(9))

    def errors(sig, x):
        out = []
        for k, l in enumerate(ls):
            ex = (2 * l + 1) * sphere.zonal_harmonic(l, x)
            out.append(rel2(sig[:, k], ex))
        return np.array(out)
    V4, T4 = icosphere(4)
    op4 = bem.Operator(V4, T4)
    F4 = np.stack([sphere.zonal_harmonic(l, op4.x) for l in ls], axis=1)
    e4 = errors(np.linalg.solve(op4.dense(), F4), op4.x)
    V, T = icosphere(6)
    x6 = bem.centroids(V, T.astype(np.int64))
    F = np.stack([sphere.zonal_harmonic(l, x6) for l in ls], axis=1)
    H = hm.HMatrix(V, T, leaf_size=64, eta=1.0, eps=1e-5, precision="f32")
    sig, info, status = H.solve(torch.tensor(F, device=DEV), tol=1e-6, restart=100, max_iter=1000)
    H.free()
    assert status == 0 and info.converged
    e6 = errors(sig.cpu().numpy(), x6)
    assert np.all(e6 <= 0.5 * e4), (e6, e4)


def test_freed_memory_cached_then_released():
    """hm_free keeps the handle's memory in the library's pool (a rebuild
    reuses it); release_memory returns it to the device."""
    import paper_1806_11558_amd as hm
    from synthetic import icosphere
    say("memory pool")
    V, T = icosphere(6)
    torch.cuda.synchronize()
    H = hm.HMatrix(V, T, leaf_size=64, eps=1e-6, precision="f64")
    held = H.stats()["device_bytes"]
    H.free()
    free_cached, _ = torch.cuda.mem_get_info()
    H = hm.HMatrix(V, T, leaf_size=64, eps=1e-6, precision="f64")   # reuses the cache
    free_rebuilt, _ = torch.cuda.mem_get_info()
    assert free_rebuilt >= free_cached - held // 4
    H.free()
    hm.release_memory()
    free_released, _ = torch.cuda.mem_get_info()
    assert free_released >= free_cached + held // 2
