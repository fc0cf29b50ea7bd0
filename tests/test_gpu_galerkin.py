"""Galerkin discretisation on the GPU (Sec. 2.2, eq. linearSystem; Sec. 4.1
and 4.3) against the Galerkin oracle: entries (singular pairs included)
element by element, every stored dense block, the products against the
dense Galerkin matrix, the partition (no admissible block holds two
triangles that share a vertex), CG against the dense LU solution, and the
harmonic test on the unit sphere whose interior error falls with h."""
import math

import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# element-wise relative tolerance of an entry.  FP64: the oracle's rules to
# rounding (the GPU sums the 49 far terms and the 144 singular terms in
# another order; its Gauss nodes come from Newton's method).  FP32 far
# entries: the centroid difference rounded to float and 49 float reciprocal
# square roots; singular entries are computed in double on both sides.
FAR_TOL = {"f64": 1e-13, "f32": 4e-6}
SING_TOL = {"f64": 1e-12, "f32": 1e-7}


@pytest.fixture(scope="module")
def gal3(ico):
    from oracle import galerkin
    V, T = ico(3)
    op = galerkin.GalerkinOperator(V, T)
    say("oracle Galerkin dense N = 1280")
    return V, T, op, op.dense()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_entries_far_and_singular(gal3, prec):
    import paper_1806_11558_amd as hm
    V, T, op, A = gal3
    say("galerkin entries", prec)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec, operator="galerkin")
    rng = np.random.default_rng(5)
    n = op.n
    rows = list(rng.integers(0, n, 300))
    cols = list(rng.integers(0, n, 300))
    sing = []
    for i in rng.integers(0, n, 60).tolist():         # self, edge and vertex neighbours
        for j in sorted(op.touching(i)):
            rows.append(i)
            cols.append(j)
            sing.append(True)
    sing = np.r_[np.zeros(300, bool), np.array(sing, bool)]
    rows, cols = np.array(rows), np.array(cols)
    got = H.entries(rows, cols)
    ref = A[rows, cols]
    err = np.abs(got - ref) / np.abs(ref)
    say("worst far", float(err[~sing].max()), "worst singular", float(err[sing].max()))
    assert err[~sing].max() <= FAR_TOL[prec]
    assert err[sing].max() <= SING_TOL[prec]
    H.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dense_blocks_every_entry(gal3, prec):
    import paper_1806_11558_amd as hm
    V, T, op, A = gal3
    say("galerkin dense blocks", prec)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec, operator="galerkin")
    perm = H.perm()
    db = H.dense_blocks()
    worst = 0.0
    for b in range(len(db)):
        r0, r1, c0, c1 = db[b, :4]
        D = H.dense_entries(b, db)
        ref = A[np.ix_(perm[r0:r1], perm[c0:c1])]
        worst = max(worst, float(np.max(np.abs(D - ref) / np.abs(ref))))
    say("worst dense entry", worst)
    assert worst <= max(FAR_TOL[prec], SING_TOL[prec])
    H.free()


def test_no_admissible_block_touches(gal3):
    """Admissible blocks of the Galerkin partition never pair triangles that
    share a vertex; every such pair is in a dense block (checked on the
    host from the mesh)."""
    import paper_1806_11558_amd as hm
    V, T, op, A = gal3
    say("galerkin partition")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, operator="galerkin")
    perm = H.perm()
    verts_of = [set(t) for t in T[perm].tolist()]
    for blk in H.lr_blocks():
        r0, r1, c0, c1 = (int(v) for v in blk[:4])
        rv = set().union(*verts_of[r0:r1])
        cv = set().union(*verts_of[c0:c1])
        assert not (rv & cv), (r0, r1, c0, c1)
    # the partition covers every entry exactly once
    d, a = H.dense_blocks(), H.lr_blocks()
    area = int(((d[:, 1] - d[:, 0]) * (d[:, 3] - d[:, 2])).sum()
               + ((a[:, 1] - a[:, 0]) * (a[:, 3] - a[:, 2])).sum())
    assert area == op.n * op.n
    # a collocation build of the same mesh may admit touching blocks; the
    # Galerkin one has at least as many dense entries
    Hc = hm.HMatrix(V, T, leaf_size=32, eps=1e-6)
    assert H.stats()["dense_entries"] >= Hc.stats()["dense_entries"]
    Hc.free()
    H.free()


@pytest.mark.parametrize("prec,eps,bound", [("f64", 1e-6, 1e-5), ("f64", 1e-8, 1e-7),
                                            ("f32", 1e-6, 1e-5)])
def test_products_vs_dense(gal3, prec, eps, bound):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = gal3
    say("galerkin products", prec, eps)
    H = hm.HMatrix(V, T, leaf_size=32, eps=eps, precision=prec, operator="galerkin")
    x = normal_columns(op.n, 3, seed=1)
    for vdt in (torch.float64, torch.float32):
        xt = torch.tensor(x, dtype=vdt, device=DEV)
        y = H.matvec(xt).double().cpu().numpy()
        yT = H.matvec_T(xt).double().cpu().numpy()
        b = bound if vdt == torch.float64 else max(bound, 1e-6)
        for k in range(3):
            assert rel2(y[:, k], A @ x[:, k]) <= b
            assert rel2(yT[:, k], A.T @ x[:, k]) <= b
    H.free()


def test_cg_vs_lu_and_gmres(gal3):
    import paper_1806_11558_amd as hm
    V, T, op, A = gal3
    say("galerkin CG")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-10, max_rank=128, operator="galerkin")
    rng = np.random.default_rng(7)
    f = np.c_[op.rhs(lambda y: 4 * y[..., 0] ** 2 - 3 * y[..., 1] ** 2 - y[..., 2] ** 2),
              rng.standard_normal(op.n)]
    ft = torch.tensor(f, device=DEV)
    s_cg, info, st = H.solve(ft, tol=1e-10, max_iter=2000, method="cg")
    assert st == hm.HM_OK, info.as_dict()
    assert info.rel_residual <= 1e-10
    s_ref = np.linalg.solve(A, f)
    s = s_cg.cpu().numpy()
    for k in range(2):
        say("CG vs LU", k, rel2(s[:, k], s_ref[:, k]), "iters", info.iters)
        assert rel2(s[:, k], s_ref[:, k]) <= 1e-6
    s_gm, info_g, st_g = H.solve(ft, tol=1e-10, method="gmres")
    assert st_g == hm.HM_OK
    assert rel2(s_gm.cpu().numpy(), s) <= 1e-8
    # float vectors in and out (the right-hand side rounded to float is the
    # system solved); the no-allocation entry point agrees bitwise
    s32, info32, st32 = H.solve(ft.float(), tol=1e-10, max_iter=2000, method="cg")
    assert st32 == hm.HM_OK
    s_ref32 = np.linalg.solve(A, ft.float().double().cpu().numpy())
    assert rel2(s32.double().cpu().numpy(), s_ref32) <= 1e-6
    sp = hm.SolveParams(tol=1e-10, restart=0, max_iter=2000, transpose=0, use_x0=0,
                        flags=hm.HM_SOLVE_CG, refine=0, inner_tol=0.0)
    s_na = torch.empty_like(ft)
    st_na, info_na = hm.hm_solve_noalloc(H._h, ft, s_na, sp)
    assert st_na == hm.HM_OK and info_na.iters == info.iters
    assert torch.equal(s_na, s_cg)
    H.free()


def test_cg_rejected_combinations(gal3):
    import paper_1806_11558_amd as hm
    V, T, op, A = gal3
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, operator="galerkin")
    ft = torch.ones(op.n, dtype=torch.float64, device=DEV)
    for kw in (dict(graph=True), dict(refine=True), dict(transpose=True)):
        with pytest.raises(hm.HMError):
            H.solve(ft, method="cg", **kw)
    H.free()


def test_interior_error_falls_with_h(ico):
    """Sec. 4.3 with the Galerkin system and CG (Sec. 4.1), N = 1,280 ..
    20,480: f = 4 x1^2 - 3 x2^2 - x3^2 on the unit sphere; the potential of
    the computed density at interior points approximates the harmonic
    extension of f, and its maximum error falls by at least 2^2.5 per
    halving of h (the paper's rate is cubic)."""
    import paper_1806_11558_amd as hm
    from oracle import galerkin
    rng = np.random.default_rng(3)
    P = rng.standard_normal((100, 3))
    P *= (0.7 * rng.random(100) ** (1.0 / 3.0) / np.linalg.norm(P, axis=1))[:, None]

    def f(y):
        return 4.0 * y[..., 0] ** 2 - 3.0 * y[..., 1] ** 2 - y[..., 2] ** 2
    eps = []
    for level in (3, 4, 5):
        V, T = ico(level)
        say("galerkin eps(h) level", level)
        op = galerkin.GalerkinOperator(V, T)
        H = hm.HMatrix(V, T, leaf_size=32, eps=1e-8, max_rank=128, operator="galerkin")
        s, info, st = H.solve(torch.tensor(op.rhs(f), device=DEV), tol=1e-8, max_iter=3000,
                              method="cg")
        assert st == hm.HM_OK
        u = galerkin.potential(V, T, s.cpu().numpy(), P)
        eps.append(float(np.max(np.abs(u - f(P)))))
        say("eps", eps[-1], "iters", info.iters)
        H.free()
    assert eps[0] > eps[1] > eps[2]
    assert math.log2(eps[0] / eps[1]) >= 2.5 and math.log2(eps[1] / eps[2]) >= 2.5


def test_fixed_rank_mode(gal3):
    """The paper's fixed-rank ACA (Sec. 4.1, rank k) on the Galerkin matrix:
    aca_eps = 0 gives every admissible block min(k, m, n) terms (k = 32 also
    runs the rerun past the first-pass cap of 24), and the product error
    against the dense Galerkin matrix falls as k grows."""
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    V, T, op, A = gal3
    x = normal_columns(op.n, 1, seed=2)[:, 0]
    ref = A @ x
    errs = []
    for k in (2, 4, 8, 32):
        say("galerkin fixed rank", k)
        H = hm.HMatrix(V, T, leaf_size=16, eta=1.0, eps=0.0, max_rank=k, operator="galerkin")
        lr = H.lr_blocks()
        cap = np.minimum(k, np.minimum(lr[:, 1] - lr[:, 0], lr[:, 3] - lr[:, 2]))
        assert np.all(lr[:, 4] <= cap) and np.mean(lr[:, 4] == cap) > 0.99
        y = H.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
        errs.append(rel2(y, ref))
        H.free()
    say("fixed-rank errors", errs)
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[3] < 1e-7


def test_batch_and_fp16_forms(ico):
    """Two meshes in one Galerkin handle (hm_build_batch: vertex indices of
    the second mesh are offset, so no pair across the meshes touches) give
    the products of the two single-mesh handles, block by block; the
    FP16-factor form at eps 1e-4 is within 10 eps of the dense Galerkin
    matrix."""
    import paper_1806_11558_amd as hm
    from oracle import galerkin
    from synthetic import normal_columns
    meshes = [ico(2), ico(3)]
    sizes = [t.shape[0] for _, t in meshes]
    x = normal_columns(sum(sizes), 2, seed=4)
    say("galerkin batch", sizes)
    Hb = hm.HMatrix.batch(meshes, leaf_size=32, eps=1e-8, operator="galerkin")
    yb = Hb.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    o = 0
    for (V, T), k in zip(meshes, sizes):
        H = hm.HMatrix(V, T, leaf_size=32, eps=1e-8, operator="galerkin")
        y = H.matvec(torch.tensor(x[o:o + k], device=DEV)).cpu().numpy()
        assert rel2(yb[o:o + k], y) <= 1e-12
        H.free()
        o += k
    Hb.free()
    V, T = ico(3)
    A = galerkin.GalerkinOperator(V, T).dense()
    say("galerkin f16")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-4, precision="f16", operator="galerkin")
    for vdt in (torch.float64, torch.float32):
        xt = torch.tensor(x[:A.shape[0]], dtype=vdt, device=DEV)
        y = H.matvec(xt).double().cpu().numpy()
        yT = H.matvec_T(xt).double().cpu().numpy()
        for k in range(2):
            assert rel2(y[:, k], A @ x[:A.shape[0], k]) <= 10 * 1e-4
            assert rel2(yT[:, k], A.T @ x[:A.shape[0], k]) <= 10 * 1e-4
    H.free()
