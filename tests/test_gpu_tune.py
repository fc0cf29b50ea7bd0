"""Autotuner (HM_AUTOTUNE): the product schedule -- every candidate unit
width is timed and the fastest kept -- and the ACA binning -- every size bin
with more than one kernel class is timed per class on a sample of its
blocks and the fastest class kept.  The tuned handle's products agree with
the untuned one's within the ACA tolerance (a bin run by another kernel
class rounds its factors differently) and with the oracle's exact rows."""
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
    # the binning: every bin with alternatives and blocks was timed per
    # class on the same sample, and the fastest class was kept
    bins, tune = H1.aca_bins(), H1.aca_tune()
    assert list(bins[:, 0]) == [64, 128, 256, 512, 1024, 2048, 4096, 2 ** 31 - 1]
    assert np.array_equal(H0.aca_bins()[:, 1], [4, 3, 2, 5, 5, 1, 1, 0])
    assert H0.aca_tune().shape == (0, 4) and len(tune) >= 2
    for b in np.unique(tune[:, 0]).astype(int):
        rows = tune[tune[:, 0] == b]
        assert len(rows) >= 2 and np.all(rows[:, 2] == rows[0, 2]) and rows[0, 2] > 0
        assert np.all(rows[:, 3] > 0)
        assert bins[b, 1] == int(rows[np.argmin(rows[:, 3]), 1])
    say("aca binning", bins[:, 1].tolist(), tune.tolist())
    x = torch.tensor(normal_columns(H0.n, 2, seed=1), device=DEV)
    for tr_ in (False, True):
        y0 = H0.matvec(x, transpose=tr_).cpu().numpy()
        y1 = H1.matvec(x, transpose=tr_).cpu().numpy()
        assert rel2(y1, y0) <= 20 * 1e-6
    # the tuned handle against exact oracle rows
    from oracle import bem
    rows = np.random.default_rng(4).choice(H0.n, 32, replace=False)
    ref = bem.Operator(V, T).matvec_rows(normal_columns(H0.n, 2, seed=1), rows)
    y1 = H1.matvec(x).cpu().numpy()[rows]
    for k in range(2):
        assert rel2(y1[:, k], ref[:, k]) <= 10 * 1e-6
    H0.free()
    H1.free()
