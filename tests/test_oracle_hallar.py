"""Pins for the oracle HALLaR solver (CPU only).

Closed-form SDP values (textbook results, Lovasz 1979 and the MaxCut SDP of
vertex-transitive graphs, (n/4) lambda_max(L)), perfect graphs theta = alpha
(Section 5.3 after eq. lovasz), brute-force bounds, a dense SDP solve on X,
exact recovery for noise-free matrix completion (Section 5.2), the
Frank-Wolfe identities (Section 2 after Alg. 1) and the invariants of
ADAP-AIPP (eq. Stationary AIPP).
"""
import math

import numpy as np
import pytest

import oracle
import sdp_instances as si
from dense_ref import brute_maxcut, brute_stable, dense_sdp

TIGHT = oracle.Options(eps=1e-7)


def _solve(prob, seed=7, opts=TIGHT):
    return oracle.hallar(prob, si.gaussian_u0(prob.n, seed), opts)


def _check(res, expected, rel=1e-6):
    assert res.status == "ok", res.status
    assert abs(res.pval - expected) <= rel * (1.0 + abs(expected)), (res.pval, expected)
    assert max(res.pinf, res.gap, res.dinf) <= 1e-7


THETA_CASES = [
    ("C5", 5, si.cycle_edges(5), math.sqrt(5.0)),
    ("C7", 7, si.cycle_edges(7), 7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7))),
    ("C8", 8, si.cycle_edges(8), 4.0),
    ("K6", 6, si.complete_edges(6), 1.0),
    ("Petersen", 10, si.petersen_edges(), 4.0),
    ("Q4", 16, si.hypercube_edges(4), 8.0),
    # 5x5 torus: edge-transitive and 4-regular, theta = -n lmin/(d - lmin), lmin = 4 cos(4 pi/5)
    ("T5x5", 25, si.torus_edges(5, 5), -25 * 4 * math.cos(4 * math.pi / 5) / (4 - 4 * math.cos(4 * math.pi / 5))),
]


@pytest.mark.parametrize("name,n,edges,theta", THETA_CASES, ids=[c[0] for c in THETA_CASES])
def test_theta_closed_forms(name, n, edges, theta):
    _check(_solve(si.theta_problem(n, *edges)), -theta)


def test_theta_empty_graph():
    """No edges (m = 0): theta = n."""
    e = np.zeros(0, np.int64)
    _check(_solve(si.theta_problem(6, e, e)), -6.0)


MAXCUT_CASES = [
    ("C5", 5, si.cycle_edges(5), 2.5 * (1 + math.cos(math.pi / 5))),
    ("C7", 7, si.cycle_edges(7), 3.5 * (1 + math.cos(math.pi / 7))),
    ("C8", 8, si.cycle_edges(8), 8.0),
    ("K6", 6, si.complete_edges(6), 9.0),
    ("Q4", 16, si.hypercube_edges(4), 32.0),
    ("T4x4", 16, si.torus_edges(4, 4), 32.0),
    ("T5x5", 25, si.torus_edges(5, 5), 25 * (1 + math.cos(math.pi / 5))),
]


@pytest.mark.parametrize("name,n,edges,val", MAXCUT_CASES, ids=[c[0] for c in MAXCUT_CASES])
def test_maxcut_closed_forms(name, n, edges, val):
    _check(_solve(si.maxcut_problem(n, *edges)), -val)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_maxcut_brute_force_bounds(seed):
    rng = np.random.default_rng(seed)
    n = 12
    i, j = si.er_edges(n, 0.4, rng)
    w = rng.uniform(0.5, 1.5, i.size)
    res = _solve(si.maxcut_problem(n, i, j, w))
    assert res.status == "ok"
    sdp = -res.pval
    mc = brute_maxcut(n, i, j, w)
    assert mc <= sdp * (1 + 1e-7)
    assert mc >= 0.878 * sdp


@pytest.mark.parametrize("seed", [0, 1])
def test_theta_brute_force_bounds(seed):
    rng = np.random.default_rng(10 + seed)
    n = 12
    i, j = si.er_edges(n, 0.35, rng)
    res = _solve(si.theta_problem(n, i, j))
    assert res.status == "ok"
    assert brute_stable(n, i, j) <= -res.pval * (1 + 1e-7)


@pytest.mark.parametrize("kind,seed", [("theta", 0), ("maxcut_pm1", 1), ("maxcut_pm1", 2)])
def test_dense_sdp_agreement(kind, seed):
    rng = np.random.default_rng(20 + seed)
    n = 9
    i, j = si.er_edges(n, 0.4, rng)
    if kind == "theta":
        prob = si.theta_problem(n, i, j)
    else:
        prob = si.maxcut_problem(n, i, j, si.pm1_weights(i.size, rng))
    pd, dd, _, _ = dense_sdp(prob)
    assert abs(pd - dd) <= 1e-7 * (1 + abs(pd))
    res = _solve(prob)
    assert res.status == "ok"
    assert abs(res.pval - pd) <= 1e-6 * (1 + abs(pd))


def test_maxcut_weak_duality_bracket():
    """Rows of U normalised give a feasible X_f; a dense eigen solve on
    C + A*(p) gives a certified dual value: dval_c <= P* <= pval_f."""
    rng = np.random.default_rng(3)
    n = 40
    i, j = si.er_edges(n, 0.15, rng)
    prob = si.maxcut_problem(n, i, j, si.pm1_weights(i.size, rng))
    res = oracle.hallar(prob, si.gaussian_u0(n, 1), oracle.Options(eps=1e-6))
    assert res.status == "ok"
    Uf = res.U / np.linalg.norm(res.U, axis=1, keepdims=True)
    pval_f = oracle.a_tilde(prob, Uf)[0]
    M = oracle.adjoint_apply(prob, np.concatenate([[1.0], res.p]), np.eye(n))
    th = max(-np.linalg.eigvalsh(M)[0], 0.0)
    dval_c = -prob.b @ res.p - prob.tau2 * th
    assert dval_c <= pval_f + 1e-12
    for v in (res.pval, res.dval):
        assert dval_c - 1e-5 * abs(dval_c) <= v <= pval_f + 1e-5 * abs(pval_f)


def test_mc_exact_recovery():
    """Noise-free completion with many samples: min Tr(X)/2 = ||M||_* ."""
    prob = si.mc_planted(30, 40, 2, 900, seed=6)
    A, B = prob.meta["A"], prob.meta["B"]
    nuc = np.linalg.svd(A @ B.T, compute_uv=False).sum()
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 2), oracle.Options(eps=1e-7))
    assert res.status == "ok"
    assert abs(res.pval - nuc) <= 1e-5 * nuc
    Y = (res.U @ res.U.T)[:30, 30:]
    assert np.linalg.norm(Y - A @ B.T) <= 1e-2 * np.linalg.norm(A @ B.T)


def test_fw_step_identity():
    """Y~ Y~^T = (1 - alpha) YY^T + alpha tau^2 y y^T (Section 2, after Alg. 1)."""
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((20, 3))
    y = rng.standard_normal(20); y /= np.linalg.norm(y)
    tau = 2.5
    for alpha in (0.0, 0.3, 0.999):
        Yt = oracle.fw_step(Y, y, 1.0, alpha, tau)
        assert Yt.shape[1] == 4
        np.testing.assert_allclose(Yt @ Yt.T, (1 - alpha) * Y @ Y.T + alpha * tau ** 2 * np.outer(y, y), atol=1e-12)
    Yt = oracle.fw_step(Y, y, 1.0, 1.0, tau)
    np.testing.assert_allclose(Yt @ Yt.T, tau ** 2 * np.outer(y, y), atol=1e-12)
    Yt = oracle.fw_step(Y, np.zeros(20), 0.0, 0.4, tau)
    np.testing.assert_allclose(Yt @ Yt.T, 0.6 * Y @ Y.T, atol=1e-12)


def test_fw_alpha_is_exact_line_search():
    """alpha minimises L_beta((1-a) YY^T + a tau^2 y y^T; p) over [0, 1]."""
    rng = np.random.default_rng(1)
    prob = si.maxcut_problem(30, *si.er_edges(30, 0.3, rng))
    Y = 0.3 * rng.standard_normal((30, 2))
    p = rng.standard_normal(30)
    beta = 2.0
    T = oracle.a_tilde(prob, Y)
    ptil = np.concatenate([[1.0], p + beta * (T[1:] - prob.b)])
    M = oracle.adjoint_apply(prob, ptil, np.eye(30))
    w, Q = np.linalg.eigh(M)
    theta, y = max(-w[0], 0.0), Q[:, 0]
    gap = float(np.sum(M * (Y @ Y.T))) + prob.tau2 * theta
    alpha = oracle.fw_alpha(gap, T[1:], oracle.a_tilde(prob, y[:, None])[1:], prob.tau2, beta)
    assert 0.0 < alpha < 1.0
    tau = math.sqrt(prob.tau2)
    f = lambda a: oracle.al_value(prob, oracle.fw_step(Y, y, theta, a, tau), p, beta)[0]
    for d in (1e-3, 1e-2):
        assert f(alpha) <= f(alpha - d) + 1e-10 and f(alpha) <= f(min(alpha + d, 1.0)) + 1e-10


def test_aipp_invariants():
    """ADAP-AIPP output: ||R|| <= rho, g(W) <= g(W_0), and R - grad g(W) lies
    in the normal cone of the Frobenius ball at W (eq. Stationary AIPP)."""
    rng = np.random.default_rng(4)
    prob = si.maxcut_problem(50, *si.er_edges(50, 0.2, rng))
    tau = math.sqrt(prob.tau2)
    p = rng.standard_normal(prob.m)
    beta = 4.0
    counters = {k: 0 for k in ("sddmm", "spmm", "fista_trials", "aipp_iters", "lam_halvings")}
    g = oracle.ALFunction(prob, p, beta, counters)
    W0 = rng.standard_normal((50, 3))
    W0 *= tau / np.linalg.norm(W0)               # start on the boundary
    g0 = g.eval(W0)[0]
    rho = 1e-4
    st, W, R, lam, gW = oracle.aipp(g, W0, g0, 1.0, rho, oracle.Options(), tau, counters)
    assert st == "ok"
    assert np.linalg.norm(W) <= tau * (1 + 1e-12)
    assert gW <= g0
    assert np.linalg.norm(R) <= rho
    N = R - oracle.al_grad(prob, W, p, beta)
    if np.linalg.norm(W) < tau * (1 - 1e-9):
        assert np.linalg.norm(N) <= 1e-8 * (1 + np.linalg.norm(R))
    else:
        c = float(np.sum(N * W)) / float(np.sum(W * W))
        assert c >= -1e-10
        assert np.linalg.norm(N - c * W) <= 1e-8 * (1 + np.linalg.norm(N))


def _capped_instance():
    rng = np.random.default_rng(0)
    i, j = si.er_edges(80, 0.1, rng)
    return si.maxcut_problem(80, i, j, si.pm1_weights(i.size, rng))


def test_rank_cap_stops_with_status():
    """A rank cap below what Frank-Wolfe asks for stops the solve with status
    "rank_cap" and the iterate before the step (rank <= cap), never silently."""
    prob = _capped_instance()
    res = oracle.hallar(prob, si.gaussian_u0(80, 3), oracle.Options(eps=1e-5, rank_cap=2))
    assert res.status == "rank_cap"
    assert res.rank <= 2
    assert res.counters["truncations"] == 0
    assert np.linalg.norm(res.U) <= math.sqrt(prob.tau2) * (1 + 1e-12)


def test_rank_cap_truncation_is_counted():
    """With truncation asked for, the cap's largest directions are kept and
    every truncation is counted."""
    prob = _capped_instance()
    res = oracle.hallar(prob, si.gaussian_u0(80, 3),
                        oracle.Options(eps=1e-5, rank_cap=2, rank_cap_truncate=True, outer_max_iter=6))
    assert res.rank <= 2
    assert res.counters["truncations"] > 0


@pytest.mark.parametrize("k1,k2,seed", [(8, 9, 1), (10, 10, 3)])
def test_certified_lambda_min_on_clustered_spectrum(k1, k2, seed):
    """+-1 tori have a cluster of smallest eigenvalues of C + A*(p) at the
    optimum (one per primal column).  The returned theta is a Ritz bound
    (theta <= max(-lambda_min, 0)) that must agree with LAPACK's lambda_min,
    and the relative gap recomputed with the exact lambda_min must meet eps
    (eq. termination2 with the exact dual value)."""
    prob = si.maxcut_torus(k1, k2, seed=seed)
    eps = 1e-5
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 7), oracle.Options(eps=eps))
    assert res.status == "ok"
    M = oracle.adjoint_apply(prob, np.concatenate([[1.0], res.p]), np.eye(prob.n))
    w = np.linalg.eigvalsh(M)
    assert w[2] - w[0] < 1e-4 * abs(w[0])           # the cluster the certification is for
    th = max(-w[0], 0.0)
    assert res.theta <= th + 1e-10
    assert th - res.theta <= 1e-6 * (1 + th)
    dval = -prob.b @ res.p - prob.tau2 * th
    assert abs(res.pval - dval) / (1 + abs(res.pval) + abs(dval)) <= eps


def test_objective_accuracy_bound():
    """With the objective test on, a converged solve also has
    |pval - dval| + |p^T r| <= eps (1 + |pval|) (the a-posteriori bound on
    the objective error); MC exact recovery (Section 5.2) then puts pval
    within eps of ||M||_* ."""
    prob = si.mc_planted(40, 50, 2, 1400, seed=8)
    A, B = prob.meta["A"], prob.meta["B"]
    nuc = np.linalg.svd(A @ B.T, compute_uv=False).sum()
    eps = 1e-5
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 3), oracle.Options(eps=eps))
    assert res.status == "ok"
    r = oracle.a_tilde(prob, res.U)[1:] - prob.b
    bound = abs(res.pval - res.dval) + abs(float(res.p @ r))
    assert bound <= eps * (1 + abs(res.pval))
    assert abs(res.pval - nuc) <= eps * (1 + nuc)


@pytest.mark.parametrize("d", [8, 10])
def test_theta_hamming_closed_form(d):
    """Lovasz theta of the Hamming graph H(d, 2) (the d-cube, Section 5.3,
    Table tab:reduced_hamming_graphs): bipartite, hence perfect, so
    theta = alpha = n/2.  The penalty has to climb to about n^2 before the
    edge constraints bind."""
    n = 1 << d
    prob = si.theta_problem(n, *si.hypercube_edges(d))
    res = oracle.hallar(prob, si.gaussian_u0(n, 5), oracle.Options(eps=1e-5))
    assert res.status == "ok"
    assert abs(res.pval + n / 2) <= 1e-5 * (1 + n / 2)
    assert max(res.pinf, res.gap, res.dinf) <= 1e-5


def test_phaselift_real_exact_recovery():
    """Real phase retrieval SDP with a rank-one low-rank term per constraint
    (the real analogue of Section 5.4): with m = 6n Gaussian measurements the
    solution is the planted x x^T, so the value is ||x||^2 (exact recovery)."""
    prob = si.phaselift_real(20, 120, seed=1)
    x = prob.meta["x"]
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 7), oracle.Options(eps=1e-6))
    assert res.status == "ok"
    assert abs(res.pval - x @ x) <= 1e-5 * (1 + x @ x)
    assert np.linalg.norm(res.U @ res.U.T - np.outer(x, x)) <= 1e-2 * (x @ x)
