"""Pins for the synthetic instance generators (CPU only): the instance
shapes the paper prints (Tables tab:gpuourmethod_vs_cpu and
tab:reduced_hamming_graphs, in tests/golden/) and structural facts of the
MaxCut / theta / matrix-completion formulations."""
import math
import os

import numpy as np
import pytest

import sdp_instances as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [list(map(int, l.split())) for l in f if l.strip() and not l.startswith("#")]


def test_mc_counts_match_paper_table():
    rows = _rows("mc_table_counts.txt")
    assert len(rows) == 22
    for n1, n2, r, m in rows:
        assert si.mc_count_tables(n1, n2, r) == m, (n1, n2, r, m)


def test_hamming_edge_counts_match_paper_table():
    for d, n, e in _rows("hamming_edges.txt"):
        assert n == 1 << d and e == n * d // 2
        if d <= 16:
            i, j = si.hypercube_edges(d)
            assert i.size == e and (i < j).all()
            assert np.unique(i * n + j).size == e


def test_er_edges_statistics():
    rng = np.random.default_rng(0)
    n, p = 3000, 0.01
    i, j = si.er_edges(n, p, rng)
    N = n * (n - 1) / 2
    assert abs(i.size - N * p) < 5 * math.sqrt(N * p)
    assert (i < j).all() and j.max() < n
    assert np.unique(i * n + j).size == i.size


def test_torus_is_4_regular():
    i, j = si.torus_edges(7, 9)
    deg = np.bincount(i, minlength=63) + np.bincount(j, minlength=63)
    assert (deg == 4).all() and i.size == 2 * 63


def test_maxcut_formulation():
    """C = -L/4 (row sums of C vanish), one diagonal constraint per vertex."""
    rng = np.random.default_rng(1)
    i, j = si.er_edges(30, 0.3, rng)
    w = si.pm1_weights(i.size, rng)
    p = si.maxcut_problem(30, i, j, w)
    C = np.zeros((30, 30))
    for a, b, l, v in zip(p.row, p.col, p.con, p.val):
        if l == 0:
            C[a, b] += v
            if a != b:
                C[b, a] += v
    np.testing.assert_allclose(C.sum(axis=1), 0.0, atol=1e-14)
    assert p.m == 30 and p.tau2 == 30.0 and (p.b == 1).all()


def test_mc_planted_point_is_feasible():
    prob = si.mc_planted(20, 30, 2, 300, seed=1)
    A, B = prob.meta["A"], prob.meta["B"]
    Z = np.vstack([A, B])
    sel = prob.con > 0
    X = Z @ Z.T
    vals = X[prob.row[sel], prob.col[sel]]
    np.testing.assert_allclose(vals, prob.b[prob.con[sel] - 1], atol=1e-12)
    assert np.trace(X) == pytest.approx(prob.tau2)


def test_served_sizes_range():
    n = si.served_stream_sizes(4096, seed=5)
    assert n.min() >= 100 and n.max() <= 20000
    assert 3000 < n.mean() < 4500
