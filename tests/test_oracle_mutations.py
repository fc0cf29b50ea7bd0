"""The pins must catch plausible mistakes: each test plants one mistake in
the oracle (on the CPU, via monkeypatch) and checks that a pin fails."""
import math

import numpy as np
import pytest

import test_oracle_aca as pins_aca
import test_oracle_cluster as pins_cluster
import test_oracle_galerkin as pins_galerkin
import test_oracle_quadrature as pins_quad
from oracle import aca, bem, cluster, galerkin, quadrature


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_wrong_quadrature_weight_is_caught(monkeypatch):
    w = quadrature.WEIGHTS.copy()
    w[1], w[4] = w[4], w[1]                       # swap the two weight groups
    monkeypatch.setattr(quadrature, "WEIGHTS", w)
    _fails(pins_quad.test_radon_rule_exact_to_degree_5, 2, 2)


def test_wrong_node_is_caught(monkeypatch):
    b = quadrature.BARY.copy()
    b[2] = b[2][[1, 0, 2]]                         # duplicate a permutation
    monkeypatch.setattr(quadrature, "BARY", b)
    _fails(pins_quad.test_radon_rule_exact_to_degree_5, 1, 0)


def test_dropped_four_pi_is_caught(monkeypatch, ico):
    monkeypatch.setattr(bem, "FOUR_PI", 1.0)
    V, T = ico(2)
    op = bem.Operator(V, T)
    # S 1 = 1 on the unit sphere fails by a factor 4 pi
    assert abs(np.mean(op.dense() @ np.ones(op.n)) - 1.0) > 1.0


def test_self_term_sign_error_is_caught(monkeypatch):
    orig = bem.self_integral

    def wrong(x, v0, v1, v2):
        return -orig(x, v0, v1, v2)
    monkeypatch.setattr(bem, "self_integral", wrong)
    _fails(pins_quad.test_self_term_equilateral_closed_form)


def test_max_instead_of_min_diameter_is_caught(monkeypatch):
    def wrong(bt, bs, eta):
        return np.maximum(cluster.diam2(bt), cluster.diam2(bs)) <= (eta * eta) * cluster.dist2(bt, bs)
    monkeypatch.setattr(cluster, "admissible", wrong)
    _fails(pins_cluster.test_admissibility_hand_boxes)


def test_transposed_morton_bits_are_caught(monkeypatch):
    orig = cluster.morton_keys

    def wrong(C):
        return orig(C[:, ::-1].copy())              # z as the most significant bit
    monkeypatch.setattr(cluster, "morton_keys", wrong)
    _fails(pins_cluster.test_morton_against_string_interleave)


def test_wrong_admissibility_in_traversal_is_caught(monkeypatch):
    orig = cluster.block_tree

    def wrong(lo, hi, child, boxes, eta, leaf):
        return orig(lo, hi, child, boxes, 2.0 * eta, leaf)   # eta applied unsquared
    monkeypatch.setattr(cluster, "block_tree", wrong)
    _fails(pins_cluster.test_partition_characterisation, 3, 32, 1.0)


def test_aca_sign_error_is_caught(monkeypatch):
    def wrong(row, col, m, n, eps, kmax):
        U, V = orig(row, col, m, n, eps, kmax)
        return U, -V
    orig = aca.aca
    monkeypatch.setattr(aca, "aca", wrong)
    _fails(pins_aca.test_exact_rank_blocks_stop_at_rank, 2)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_galerkin_dropped_height_terms_are_caught(monkeypatch):
    """The off-plane part of the closed-form inner integral left out."""
    monkeypatch.setattr(galerkin, "_height_terms", lambda ad, h, la, lb, ra, rb: 0.0 * ad)
    _fails(pins_galerkin.test_inner_integral_off_plane_matches_brute_force)


def test_galerkin_unsigned_sub_triangles_are_caught(monkeypatch):
    """Every sub-triangle counted positive (a point beyond an edge then
    over-counts): an in-plane point outside T and the touching pairs."""
    monkeypatch.setattr(galerkin, "_signed", lambda cr, val: val)
    _fails(pins_galerkin.test_inner_integral_off_plane_matches_brute_force)


def test_galerkin_dropped_four_pi_is_caught(monkeypatch, ico):
    monkeypatch.setattr(galerkin, "FOUR_PI", 1.0)
    # both rules scale alike (their comparison cannot see it); the harmonic
    # test on the sphere does
    _fails(pins_galerkin.test_interior_error_third_order_on_the_unit_sphere, ico)
