"""GMRES with one replayed HIP graph per Arnoldi step (HM_SOLVE_GRAPH):
every replay, interleaved with eager products, solves and host
synchronisations, gives bitwise the result of the eager solve."""
import numpy as np
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("prec,level", [("f32", 4), ("f64", 3), ("f16", 4)])
def test_graph_solves_match_eager(prec, level):
    import paper_1806_11558_amd as hm
    from synthetic import icosphere, normal_columns
    say("graph solve", prec, level)
    V, T = icosphere(level)
    H = hm.HMatrix(V, T, leaf_size=32, eps=1e-6, precision=prec)
    n = H.n
    for nrhs, transpose in [(1, False), (3, False), (1, True), (3, False)]:
        F = normal_columns(n, nrhs, seed=nrhs + 10 * transpose)
        f = torch.tensor(F[:, 0] if nrhs == 1 else F, device=DEV)
        ref, info_ref, st_ref = H.solve(f, tol=1e-9, restart=30, transpose=transpose)
        ref = ref.cpu().numpy()
        for rep in range(3):
            # eager work between the replays
            _ = H.matvec(f)
            torch.cuda.synchronize()
            got, info, st = H.solve(f, tol=1e-9, restart=30, transpose=transpose, graph=True)
            assert st == st_ref and info.iters == info_ref.iters
            assert np.array_equal(got.cpu().numpy(), ref), (nrhs, transpose, rep)
    H.free()
