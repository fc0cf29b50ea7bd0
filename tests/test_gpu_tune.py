"""Product-schedule autotuner (HM_AUTOTUNE): every candidate width is timed,
the fastest is kept, and the tuned handle's products agree with the
untuned one's to rounding (only the order of partial-row sums differs)."""
import numpy as np
import pytest
import torch

from gpu_util import rel2, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("prec,level,leaf", [("f64", 4, 32), ("f32", 6, 64)])
def test_autotune_picks_fastest_and_keeps_results(prec, level, leaf):
    import paper_1806_11558_amd as hm
    from synthetic import icosphere, normal_columns
    say("autotune", prec, level)
    V, T = icosphere(level)
    H0 = hm.HMatrix(V, T, leaf_size=leaf, eps=1e-6, precision=prec)
    H1 = hm.HMatrix(V, T, leaf_size=leaf, eps=1e-6, precision=prec, autotune=True)
    tr = H1.tune_results()
    assert tr.shape == (5, 2) and np.all(tr[:, 1] > 0)
    assert list(tr[:, 0]) == [512, 1024, 2048, 4096, 8192]
    assert H1.stats()["unit_cols"] == int(tr[np.argmin(tr[:, 1]), 0])
    assert H0.stats()["unit_cols"] == 1024 and H0.tune_results().shape == (0, 2)
    x = torch.tensor(normal_columns(H0.n, 2, seed=1), device=DEV)
    for tr_ in (False, True):
        y0 = H0.matvec(x, transpose=tr_).cpu().numpy()
        y1 = H1.matvec(x, transpose=tr_).cpu().numpy()
        assert rel2(y1, y0) <= (1e-14 if prec == "f64" else 1e-12)
    H0.free()
    H1.free()
