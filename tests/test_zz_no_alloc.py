"""hm_solve_noalloc: the solve with its workspace in the library's fixed
device array.  Same stored operator, same kernels and order as hm_solve, so
the solution and the reported info must be bitwise those of hm_solve; two
calls in a row (the second on a smaller system) check that nothing is
carried over from the previous call; oversized requests and the graph flag
are refused before any device work."""
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _both(H, f, **kw):
    import paper_1806_11558_amd as hm
    sp = hm.SolveParams(tol=kw.get("tol", 1e-8), restart=kw.get("restart", 40),
                        max_iter=kw.get("max_iter", 2000),
                        transpose=1 if kw.get("transpose") else 0, use_x0=0, flags=0,
                        refine=1 if kw.get("refine") else 0, inner_tol=kw.get("inner_tol", 0.0))
    s_ref = torch.empty_like(f)
    st_ref, info_ref = hm.hm_solve(H._h, f, s_ref, sp)
    s = torch.full_like(f, float("nan"))
    st, info = hm.hm_solve_noalloc(H._h, f, s, sp)
    torch.cuda.synchronize()
    return (s_ref, st_ref, info_ref), (s, st, info)


def _same(a, b):
    (s_ref, st_ref, i_ref), (s, st, i) = a, b
    assert st == st_ref
    assert (i.iters, i.restarts, i.converged, i.ir_steps) == \
        (i_ref.iters, i_ref.restarts, i_ref.converged, i_ref.ir_steps)
    assert i.rel_residual == i_ref.rel_residual
    assert torch.equal(s, s_ref)


def test_noalloc_solve_matches_solve_twice(ico):
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns
    # first call: N = 1,280, three right-hand sides, refined FP32 form
    V, T = ico(3)
    say("noalloc: N = 1280, f32, 3 rhs, refine")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision="f32")
    f = torch.tensor(normal_columns(T.shape[0], 3, seed=21), device=DEV)
    a, b = _both(H, f, refine=True, inner_tol=1e-4)
    _same(a, b)
    assert b[1] == hm.HM_OK and b[2].ir_steps >= 2
    # plain double GMRES, transposed, same handle
    say("noalloc: N = 1280, f32, transposed, plain")
    _same(*_both(H, f[:, :1].contiguous(), transpose=True))
    H.free()
    # second call: a smaller system (N = 320, one column, FP64 form)
    V2, T2 = ico(2)
    say("noalloc: N = 320, f64, 1 rhs")
    H2 = hm.HMatrix(V2, T2, leaf_size=16, eps=1e-8, precision="f64")
    f2 = torch.tensor(normal_columns(T2.shape[0], 1, seed=22)[:, 0], device=DEV)
    a2, b2 = _both(H2, f2, tol=1e-10)
    _same(a2, b2)
    assert b2[1] == hm.HM_OK
    H2.free()


def test_noalloc_rejects_oversized_and_graph(ico):
    import paper_1806_11558_amd as hm
    V, T = ico(3)
    say("noalloc: rejections")
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision="f32")
    n = T.shape[0]
    # 8 * (1000 + 7) * 1280 * 64 bytes = 660 MB > the fixed 128 MiB
    f = torch.ones((n, 64), dtype=torch.float64, device=DEV)
    s = torch.zeros_like(f)
    sp = hm.SolveParams(tol=1e-8, restart=1000, max_iter=10, transpose=0, use_x0=0, flags=0,
                        refine=0, inner_tol=0.0)
    with pytest.raises(hm.HMError) as e:
        hm.hm_solve_noalloc(H._h, f, s, sp)
    assert e.value.status == hm.HM_ERR_ARG and "bytes" in str(e.value)
    assert torch.count_nonzero(s).item() == 0
    sp = hm.SolveParams(tol=1e-8, restart=30, max_iter=10, transpose=0, use_x0=0,
                        flags=hm.HM_SOLVE_GRAPH, refine=0, inner_tol=0.0)
    with pytest.raises(hm.HMError) as e:
        hm.hm_solve_noalloc(H._h, f[:, :1].contiguous(), s[:, :1].contiguous(), sp)
    assert e.value.status == hm.HM_ERR_ARG
    H.free()
