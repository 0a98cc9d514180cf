"""GPU parity of the full HALLaR solve (hallar_solve) in FP64 and FP32-mixed.

Final objectives are compared with closed-form SDP values (Lovasz theta and
MaxCut of vertex-transitive graphs) and with FP64 oracle solves at
eps = 1e-7 (1e-6 for the torus) stored in tests/golden/refs.json (written by
make_refs.py, which calls only the oracle).  Bar, in both precisions:
|pval - ref| <= 1e-5 (1 + |ref|), with the solve's relative gap,
infeasibility and dual infeasibility <= its eps.  Both solvers stop only when
the a-posteriori objective bound |pval - dval| + |p^T (A(X) - b)| is within
eps (1 + |pval|) as well (the relative gap of eq. termination2 divides by
about twice the objective, so alone it admits an objective error near
2 eps), which is what lets a solve at eps = 1e-5 meet the 1e-5 objective bar.
"""
import json
import math
import os

import numpy as np
import pytest

import sdp_instances as si
from gpu_util import dev, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu

REFS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "refs.json"))) \
    if os.path.exists(os.path.join(os.path.dirname(__file__), "golden", "refs.json")) else {}


def solve(prob, prec=H.FP64, eps=1e-5, seed=7, **kw):
    d = dev()
    h = H.hallar_create(prob, prec, H.options(eps=eps, **kw))
    try:
        U0 = torch.tensor(si.gaussian_u0(prob.n, seed), device=d)
        res = H.hallar_solve(h, U0)
        U = torch.empty((prob.n, max(res["rank"], 1)), dtype=torch.float64, device=d)
        p = torch.empty(max(prob.m, 1), dtype=torch.float64, device=d)
        H.hallar_get_solution(h, U, p)
        return res, U.cpu().numpy(), p.cpu().numpy()[: prob.m]
    finally:
        H.hallar_destroy(h)


def check(res, ref, eps, rel=1e-5):
    assert res["status"] == "ok", res
    assert max(res["pinf"], res["gap"], res["dinf"]) <= eps
    assert abs(res["pval"] - ref) <= rel * (1.0 + abs(ref)), (res["pval"], ref)


CLOSED = [
    ("theta_C5", si.theta_problem(5, *si.cycle_edges(5)), -math.sqrt(5.0)),
    ("theta_petersen", si.theta_problem(10, *si.petersen_edges()), -4.0),
    ("theta_Q4", si.theta_problem(16, *si.hypercube_edges(4)), -8.0),
    ("maxcut_C5", si.maxcut_problem(5, *si.cycle_edges(5)), -2.5 * (1 + math.cos(math.pi / 5))),
    ("maxcut_K6", si.maxcut_problem(6, *si.complete_edges(6)), -9.0),
    ("maxcut_T5x5", si.maxcut_problem(25, *si.torus_edges(5, 5)), -25 * (1 + math.cos(math.pi / 5))),
    ("maxcut_T8x8_unit", si.maxcut_torus(8, 8, unit=True), -128.0),
]


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED])
@pytest.mark.parametrize("name,prob,val", CLOSED, ids=[c[0] for c in CLOSED])
def test_closed_forms(prec, name, prob, val):
    # FP64 at eps = 1e-6, FP32-mixed at the 1e-5 of its bar; both within
    # 1e-5 relative of the closed form
    eps = 1e-6 if prec == H.FP64 else 1e-5
    res, U, p = solve(prob, prec, eps=eps)
    check(res, val, eps)
    assert np.linalg.norm(U) <= math.sqrt(prob.tau2) * (1 + 1e-6)     # U stays in B_tau


def test_solution_is_consistent():
    """The returned U reproduces pval; p satisfies dval = -b^T p - tau^2 theta."""
    import oracle
    prob = si.maxcut_problem(40, *si.er_edges(40, 0.2, np.random.default_rng(1)))
    res, U, p = solve(prob, H.FP64, eps=1e-6)
    assert res["status"] == "ok"
    assert abs(oracle.a_tilde(prob, U)[0] - res["pval"]) <= 1e-9 * (1 + abs(res["pval"]))
    assert abs(-prob.b @ p - prob.tau2 * res["theta"] - res["dval"]) <= 1e-9 * (1 + abs(res["dval"]))


REF_CASES = [
    # the r <= 16 cap is met by truncation (opts.rank_cap_truncate), the final
    # certificate judging the result; the strict cap is tested below
    ("maxcut_er800_s1", lambda: si.maxcut_er_800(1), dict(rank_cap=16, rank_cap_truncate=1)),
    ("maxcut_pm1_er400", None, {}),
    ("torus_pm1_20x20", lambda: si.maxcut_torus(20, 20, seed=3), {}),
    ("theta_er150", None, {}),
    ("mc_60x90", lambda: si.mc_planted(60, 90, 2, 2500, seed=6), {}),
]


def _make(name, maker):
    if maker is not None:
        return maker()
    if name == "maxcut_pm1_er400":
        rng = np.random.default_rng(11)
        i, j = si.er_edges(400, 0.02, rng)
        return si.maxcut_problem(400, i, j, si.pm1_weights(i.size, rng))
    rng = np.random.default_rng(12)
    i, j = si.er_edges(150, 0.06, rng)
    return si.theta_problem(150, i, j)


def objective_bound(prob, res, U, p):
    """|pval - dval| + |p^T (A(X) - b)|: with the dual iterate feasible up to
    dinf, dval <= P* <= pval + |p^T r|, so this bounds |pval - P*|."""
    import oracle
    r = oracle.a_tilde(prob, U)[1:] - prob.b
    return abs(res["pval"] - res["dval"]) + abs(float(p @ r))


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED])
@pytest.mark.parametrize("name,maker,kw", REF_CASES, ids=[c[0] for c in REF_CASES])
def test_against_oracle_reference(prec, name, maker, kw):
    if name not in REFS:
        pytest.skip("tests/golden/refs.json lacks " + name)
    ref = REFS[name]
    assert ref["status"] == "ok", ref
    if name == "theta_er150" and prec == H.FP32_MIXED:
        # measured: iteration limit with relative gap 1.7e-4 (beta 2.6e5).
        # The edge constraints ask X_ij = <U_i, U_j> = 0 of rows stored in
        # FP32, whose rounding (~u |U_i||U_j|) sits at the scale of the
        # steps ADAP-FISTA has to take near the optimum: the FP32-mixed form
        # does not reach eps = 1e-5 on this Lovasz theta instance
        pytest.xfail("FP32-mixed theta on G(150, 0.06): iteration limit at gap 1.7e-4")
    prob = _make(name, maker)
    res, U, p = solve(prob, prec, eps=1e-5, **kw)
    check(res, ref["pval"], 1e-5)
    # the reported objective bound is the one recomputed from U and p
    assert abs(res["obj_bound"] - objective_bound(prob, res, U, p)) <= 1e-6 * (1.0 + abs(res["pval"]))
    assert res["obj_bound"] <= 1e-5 * (1.0 + abs(res["pval"]))


def test_objective_check_off_admits_larger_error():
    """With opts.obj_check = 0 only the three relative errors stop the solve;
    the reported bound then exceeds eps (1 + |pval|) on the +-1 MaxCut
    instance, and turning the check on brings the objective within 1e-5."""
    name = "maxcut_pm1_er400"
    if name not in REFS:
        pytest.skip("no reference")
    prob = _make(name, None)
    ref = REFS[name]["pval"]
    off, _, _ = solve(prob, H.FP64, eps=1e-5, obj_check=0)
    on, _, _ = solve(prob, H.FP64, eps=1e-5)
    assert off["status"] == on["status"] == "ok"
    assert on["outer_iters"] >= off["outer_iters"]
    assert abs(on["pval"] - ref) <= 1e-5 * (1 + abs(ref))
    assert abs(off["pval"] - ref) <= off["obj_bound"] + 1e-7 * abs(ref)


def test_rank_cap_status_matches_oracle():
    """Reading R13: a Frank-Wolfe step over the rank cap stops the solve with
    E_RANK_CAP on the GPU and "rank_cap" in the oracle, returning the iterate
    before the step (rank <= cap); with rank_cap_truncate the GPU keeps the
    cap's largest directions and counts each truncation."""
    import oracle
    rng = np.random.default_rng(0)
    i, j = si.er_edges(80, 0.1, rng)
    prob = si.maxcut_problem(80, i, j, si.pm1_weights(i.size, rng))
    ores = oracle.hallar(prob, si.gaussian_u0(80, 7), oracle.Options(eps=1e-5, rank_cap=2))
    assert ores.status == "rank_cap"
    for prec in (H.FP64, H.FP32_MIXED):
        res, U, _ = solve(prob, prec, eps=1e-5, rank_cap=2)
        assert res["status"] == "rank_cap", res
        assert res["rank"] <= 2 and res["n_truncations"] == 0
        assert np.linalg.norm(U) <= math.sqrt(prob.tau2) * (1 + 1e-6)
        tr, _, _ = solve(prob, prec, eps=1e-5, rank_cap=2, rank_cap_truncate=1, outer_max_iter=6)
        assert tr["rank"] <= 2 and tr["n_truncations"] > 0


def test_autotuned_schedule_solves_alike():
    """opts.autotune = 1 picks one of the candidate tile schedules by timing
    the SDDMM and SpMM entry points; the solve agrees with the default
    schedule's to the solve tolerance (partial-sum order differs)."""
    d = dev()
    prob = si.mc_planted(300, 400, 2, 20000, seed=8)
    res = {}
    for tune in (0, 1):
        h = H.hallar_create(prob, H.FP32_MIXED, H.options(eps=1e-5, autotune=tune))
        try:
            mr, cap, nt = H.hallar_schedule(h)
            assert (mr, cap) in [(64, 2048), (16, 2048), (256, 2048), (64, 1024), (16, 512), (256, 1024)]
            if not tune:
                assert (mr, cap) == (64, 2048)
            assert nt >= 1
            res[tune] = H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, 7), device=d))
        finally:
            H.hallar_destroy(h)
    for r in res.values():
        assert r["status"] == "ok", r
    assert abs(res[0]["pval"] - res[1]["pval"]) <= 1e-5 * (1 + abs(res[0]["pval"]))


LOWER_CASES = [
    ("mc_300x400", lambda: si.mc_planted(300, 400, 2, 20000, seed=8), H.FP32_MIXED, 1, True),
    ("mc_300x400_fp64", lambda: si.mc_planted(300, 400, 2, 20000, seed=8), H.FP64, 1, True),
    # low-rank objective term: recomputed lower half, never fused
    ("theta_er150", lambda: _make("theta_er150", None), H.FP64, 1, False),
    # a 12-column start: 16-column FP32 rows, four lanes per row (butterfly
    # dots), fused only once the rank falls to 8 or less
    ("mc_wide_fp32", lambda: si.mc_planted(200, 300, 6, 15000, seed=9), H.FP32_MIXED, 12, None),
]


@pytest.mark.parametrize("name,maker,prec,r0,fused", LOWER_CASES, ids=[c[0] for c in LOWER_CASES])
def test_lower_recompute_and_fusion_bitwise(name, maker, prec, r0, fused):
    """The gradient SpMM's lower half recomputed from the factor rows and
    (p_l, b_l) in lower order (opts.lower_gather = 0) takes the SDDMM's
    arithmetic, so that solve is bit-identical to the gathering one.  The
    fused trial kernel (opts.unfused_trial = 0) forms the same pair values
    and SpMM sums but adds the SDDMM's partial sums in walk order, so its
    solve agrees to the solve tolerance.  The profile tells the paths apart:
    the SpMM's algorithmic bytes (column + (p_l, b_l) vs column + pair id)
    and the fused kernel's launches."""
    d = dev()
    prob = maker()
    out = {}
    for cfg in ((1, 1), (0, 1), (0, 0)):
        lg, uf = cfg
        h = H.hallar_create(prob, prec, H.options(eps=1e-5, profile=1, lower_gather=lg, unfused_trial=uf))
        try:
            U_0 = np.random.default_rng(7).standard_normal((prob.n, r0))
            res = H.hallar_solve(h, torch.tensor(U_0, device=d))
            U = torch.empty((prob.n, max(res["rank"], 1)), dtype=torch.float64, device=d)
            p = torch.empty(max(prob.m, 1), dtype=torch.float64, device=d)
            H.hallar_get_solution(h, U, p)
            out[cfg] = (res, U.cpu().numpy(), p.cpu().numpy(), H.hallar_profile(h))
        finally:
            H.hallar_destroy(h)
    r1, U1, p1, f1 = out[(1, 1)]
    assert r1["status"] == "ok", r1
    r0_, U0_, p0_, _ = out[(0, 1)]
    for k in ("pval", "dval", "gap", "pinf", "rank", "outer_iters", "n_fista_trials", "n_spmm", "n_hlr_iters"):
        assert r0_[k] == r1[k], (k, r0_[k], r1[k])
    assert np.array_equal(U0_, U1) and np.array_equal(p0_, p1)
    rf = out[(0, 0)][0]
    assert rf["status"] == "ok", rf
    assert max(rf["pinf"], rf["gap"], rf["dinf"]) <= 1e-5
    assert abs(rf["pval"] - r1["pval"]) <= 1e-5 * (1 + abs(r1["pval"])), (rf["pval"], r1["pval"])
    assert out[(0, 1)][3]["spmm"]["bytes"] != f1["spmm"]["bytes"]
    assert out[(0, 1)][3]["sddmm_spmm"]["launches"] == 0 and f1["sddmm_spmm"]["launches"] == 0
    nf = out[(0, 0)][3]["sddmm_spmm"]["launches"]
    if fused is True:
        assert nf > 0
    elif fused is False:
        assert nf == 0


def test_profile_levels():
    """opts.profile = 1 times every kernel class, 2 only the sparse ones (SDDMM,
    SpMM, fused trial, Lanczos SpMV), 0 none; the solve is the same at every
    level (the events do not touch the data)."""
    d = dev()
    prob = si.mc_planted(300, 400, 2, 20000, seed=8)
    out = {}
    for level in (0, 1, 2):
        h = H.hallar_create(prob, H.FP32_MIXED, H.options(eps=1e-5, profile=level))
        try:
            res = H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, 7), device=d))
            out[level] = (res, H.hallar_profile(h))
        finally:
            H.hallar_destroy(h)
    sparse = ("sddmm", "spmm", "lanczos_spmv", "sddmm_spmm")
    for k, v in out[0][1].items():
        assert v["launches"] == 0 and v["ms"] == 0.0, k
    assert all(out[1][1][k]["launches"] > 0 for k in ("vector", "reduce", "sddmm_spmm"))
    for k, v in out[2][1].items():
        if k in sparse:
            assert v["launches"] == out[1][1][k]["launches"], k
        else:
            assert v["launches"] == 0, k
    assert out[0][0]["pval"] == out[1][0]["pval"] == out[2][0]["pval"]


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED])
def test_repeated_solves_identical(prec):
    """A solve depends on the instance, U0 and the options only: repeated
    solves on one handle, with an eigen solve on other multipliers in
    between, give the same bits (nothing of an earlier solve or call, such as
    the last Lanczos shift, carries over); repeated eigen solves agree too."""
    d = dev()
    rng = np.random.default_rng(3)
    i, j = si.er_edges(500, 8.0 / 499, rng)
    prob = si.maxcut_problem(500, i, j, si.pm1_weights(i.size, rng))
    h = H.hallar_create(prob, prec, H.options(eps=1e-5))
    try:
        U0 = torch.tensor(si.gaussian_u0(prob.n, 7), device=d)
        out = []
        for k in range(3):
            res = H.hallar_solve(h, U0)
            U = torch.empty((prob.n, res["rank"]), dtype=torch.float64, device=d)
            H.hallar_get_solution(h, U, None)
            out.append((res, U.cpu()))
            if k == 0:
                v = torch.empty(prob.n, dtype=torch.float64, device=d)
                p = torch.tensor(rng.standard_normal(prob.m), device=d)
                lams = [H.hallar_min_eig(h, p, v, tol=1e-9, max_iter=40)[0] for _ in range(2)]
                assert lams[0] == lams[1]
        for res, U in out[1:]:
            for k in ("status", "pval", "dval", "gap", "rank", "n_fista_trials", "n_matvec", "n_rounds"):
                assert res[k] == out[0][0][k], (k, res[k], out[0][0][k])
            assert torch.equal(U, out[0][1])
    finally:
        H.hallar_destroy(h)
