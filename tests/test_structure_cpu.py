"""Host-side structure of an instance (hallar_inspect, no GPU): the union
support S and the pattern S u S^T (Section 4.1), the mode flags that choose
the kernels' fast paths, and the tile schedule.  Pair counts and row degrees
are recomputed here from the problem's triplets with numpy."""
import numpy as np
import pytest

import sdp_instances as si
from paper_2505_13719_amd import hallar as H

TILE_ROWS, TILE_ENTRIES = 1024, 2048


def _support(prob):
    key = np.unique(prob.row.astype(np.int64) * prob.n + prob.col.astype(np.int64))
    i, j = key // prob.n, key % prob.n
    deg = np.bincount(i, minlength=prob.n) + np.bincount(j[i != j], minlength=prob.n)
    return i, j, deg


FAMILIES = [
    # name, problem, direct, constraint rule, lower half recomputed
    ("matrix_completion", lambda: si.mc_planted(300, 400, 2, 60000, seed=8), 1, 1, 1),
    ("maxcut_er", lambda: si.maxcut_problem(60, *si.er_edges(60, 0.2, np.random.default_rng(1))), 1, 2, 0),
    ("maxcut_torus", lambda: si.maxcut_torus(8, 8, unit=True), 1, 2, 0),
    ("theta", lambda: si.theta_problem(10, *si.petersen_edges()), 1, 1, 1),
    ("general_hslr", lambda: si.random_hslr(8, 4, 0), 0, 0, 0),
]


@pytest.mark.parametrize("name,maker,direct,rule,lowrec", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_modes_and_pair_counts(name, maker, direct, rule, lowrec):
    prob = maker()
    d = H.hallar_inspect(prob)
    i, j, _ = _support(prob)
    assert d["pairs"] == i.size
    assert d["lower"] == int((i != j).sum())
    assert (d["direct"], d["con_rule"], d["lower_recompute"]) == (direct, rule, lowrec)


def test_mixed_constraint_pattern_has_no_rule():
    """MaxCut plus one constrained off-diagonal pair: neither 'exactly the
    diagonal' nor 'exactly the off-diagonal pairs' is constrained, and the
    other off-diagonal pairs carry no constraint, so the lower half cannot be
    recomputed from (p_l, b_l)."""
    prob = si.maxcut_problem(30, *si.er_edges(30, 0.3, np.random.default_rng(2)))
    off = np.flatnonzero(prob.row != prob.col)[0]
    con = prob.con.copy()
    m = prob.m + 1
    con[off] = m
    q = si.Problem(name="maxcut_mixed", n=prob.n, m=m, tau2=prob.tau2, row=prob.row, col=prob.col, con=con, val=prob.val,
                   b=np.append(prob.b, 0.0))
    d = H.hallar_inspect(q)
    assert d["direct"] == 1 and d["con_rule"] == 0 and d["lower_recompute"] == 0


@pytest.mark.parametrize("maker", [lambda: si.mc_planted(300, 400, 2, 60000, seed=8),
                                   lambda: si.mc_planted(2000, 1500, 2, 150000, seed=3),
                                   lambda: si.maxcut_torus(100, 100, unit=True),
                                   lambda: si.theta_er(3000, 10.0, seed=1)],
                         ids=["mc_long_rows", "mc_medium_rows", "torus_short_rows", "theta_er"])
def test_tile_schedule(maker):
    """Tiles cover the rows in order; each holds at most 1024 rows and 2048
    entries of S u S^T unless it is a single row; a tile closed by the entry
    cap (the next row did not fit) with 4..128 rows has a power-of-two row
    count, so the SpMM's power-of-two row teams fill the workgroup."""
    prob = maker()
    _, _, deg = _support(prob)
    r = H.hallar_inspect(prob)["tile_row0"]
    assert r[0] == 0 and r[-1] == prob.n and (np.diff(r) > 0).all()
    cum = np.concatenate([[0], np.cumsum(deg)])
    row_target = min(TILE_ROWS, max(64, -(-prob.n // 2048)))
    for t in range(r.size - 1):
        r0, r1 = int(r[t]), int(r[t + 1])
        rows, ent = r1 - r0, int(cum[r1] - cum[r0])
        assert rows <= TILE_ROWS
        assert ent <= TILE_ENTRIES or rows == 1
        if r1 < prob.n and rows < row_target:
            # closed before the row target: by the entry cap, and cut to a power of two
            if 4 <= rows <= 128:
                assert rows & (rows - 1) == 0, (t, rows)
            # the rows up to the next power of two would not have fitted
            nxt = min(prob.n, r0 + 2 * rows)
            assert rows < 4 or int(cum[nxt] - cum[r0]) > TILE_ENTRIES or nxt - r0 > row_target
