"""The per-outer-iteration records of a solve (hallar_get_history): one per
outer iteration, the last one equal to the result's quantities, counters
cumulative, and a batched solve's records equal to the same solve alone
(apart from the clock)."""
import numpy as np
import pytest

import sdp_instances as si
from gpu_util import dev, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu

SAME = ("t", "rank", "beta", "pval", "dval", "theta", "pinf", "gap", "dinf", "obj_bound", "n_fista_trials",
        "n_matvec", "n_hlr_iters")


def _probs():
    rng = np.random.default_rng(8)
    i, j = si.er_edges(400, 8.0 / 399, rng)
    return [si.maxcut_problem(5, *si.cycle_edges(5)), si.maxcut_problem(400, i, j, si.pm1_weights(i.size, rng)),
            si.theta_problem(10, *si.petersen_edges())]


def test_history_matches_result():
    d = dev()
    for prob in _probs():
        h = H.hallar_create(prob, H.FP64, H.options(eps=1e-6))
        try:
            res = H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, 3), device=d))
            hist = H.hallar_get_history(h)
        finally:
            H.hallar_destroy(h)
        assert res["status"] == "ok"
        assert len(hist) == res["outer_iters"] >= 1
        assert [r["t"] for r in hist] == list(range(1, len(hist) + 1))
        last = hist[-1]
        for k in ("pval", "dval", "theta", "pinf", "gap", "dinf", "rank", "beta", "obj_bound", "n_fista_trials",
                  "n_matvec", "n_hlr_iters"):
            assert last[k] == res[k], (k, last[k], res[k])
        assert max(last["pinf"], last["gap"], last["dinf"]) <= 1e-6
        for a, b in zip(hist, hist[1:]):
            assert b["beta"] >= a["beta"] and b["seconds"] >= a["seconds"]
            for k in ("n_fista_trials", "n_matvec", "n_hlr_iters"):
                assert b[k] >= a[k]


def test_history_batched_equals_alone():
    d = dev()
    probs = _probs()
    alone = []
    for prob in probs:
        h = H.hallar_create(prob, H.FP64, H.options(eps=1e-6))
        try:
            H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, 3), device=d))
            alone.append(H.hallar_get_history(h))
        finally:
            H.hallar_destroy(h)
    hs = [H.hallar_create(p, H.FP64, H.options(eps=1e-6)) for p in probs]
    try:
        H.hallar_solve_batch(hs, [torch.tensor(si.gaussian_u0(p.n, 3), device=d) for p in probs])
        batched = [H.hallar_get_history(h) for h in hs]
    finally:
        for h in hs:
            H.hallar_destroy(h)
    for a, b in zip(alone, batched):
        assert len(a) == len(b)
        for ra, rb in zip(a, b):
            for k in SAME:
                assert ra[k] == rb[k], (k, ra[k], rb[k])
