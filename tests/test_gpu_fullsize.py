"""Parity at the full sizes the benchmark runs, in the launch configuration it
times (FP32-mixed, default tile schedule):

* the matrix-completion SDP c3 (n1 = n2 = 1e5, rank 3, m = 1.2e7 observed
  entries) and the +-1 torus 1000 x 1000 (n = 1e6, r = 32): the operator
  entry points (eq. A tilde operator, Algorithms 2-5) against the FP64 oracle
  on every output -- the oracle's vectorised operators finish in seconds at
  these sizes -- with the FP32-mixed bar of the small-instance tests;
* the full c3 solve in FP64 and FP32-mixed, the path the benchmark times
  (fused trial kernel, split reductions, recomputed lower half): its
  objective is within 1e-5 of the closed-form optimum ||A B^T||_* (exact
  recovery, Section 5.2), and its certificate is recomputed
  independently of the GPU -- the oracle evaluates C . UU^T and
  A(UU^T) - b from the returned U (eq. termination2), and scipy's eigsh
  computes lambda_min(C + A*(p)) for the dual value -b^T p -
  tau^2 max(-lambda_min, 0).

The solver's gap, like the paper's criterion, uses the eigensolver's
smallest Ritz value, an upper bound on lambda_min.  Near the optimum of this
SDP the smallest eigenvalues of C + A*(p) form a cluster (one per column of
the rank-3 primal solution), and a warm-started Lanczos run can settle on a
cluster member above the minimum (theta 0.006239 against eigsh's 0.006255,
exact gap 1.22e-5 where 3.95e-6 was reported).  The solver therefore
confirms convergence with a cold-started run; the test pins the Ritz bound
(theta never above the exact value) and the exact gap within eps.
"""
import functools

import numpy as np
import pytest

import oracle
import sdp_instances as si
from gpu_util import U32, U64, abs_terms_T, abs_terms_W, dev, entrywise, normwise, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


@functools.lru_cache(maxsize=None)
def _instance(name):
    if name == "mc_1e5x1e5_r3":
        n1 = n2 = 100_000
        return si.mc_planted(n1, n2, 3, 20 * 3 * (n1 + n2), seed=4)
    return si.maxcut_torus(1000, 1000, seed=2)


@pytest.mark.parametrize("name,r", [("mc_1e5x1e5_r3", 3), ("torus_1000x1000", 32)])
def test_fullsize_operators(name, r):
    d = dev()
    prob = _instance(name)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((prob.n, r)).astype(np.float32)
    p = rng.standard_normal(prob.m)
    print(f"[fullsize] {name}: n={prob.n} m={prob.m} r={r}", flush=True)
    h = H.hallar_create(prob, H.FP32_MIXED)
    try:
        Ud = torch.tensor(U, device=d)
        T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
        H.hallar_eval_AUUt(h, Ud, T)
        pd = torch.tensor(p, dtype=torch.float64, device=d)
        W = torch.empty((prob.n, r), dtype=torch.float32, device=d)
        H.hallar_adjoint_spmm(h, pd, Ud, W)
        torch.cuda.synchronize()
        T, W = T.cpu().numpy(), W.double().cpu().numpy()
    finally:
        H.hallar_destroy(h)
    Uo = U.astype(np.float64)  # the exact values the GPU multiplied
    Tref, tT = oracle.a_tilde(prob, Uo), abs_terms_T(prob, Uo)
    assert normwise(T, Tref, tT) <= TOL_FP32
    assert entrywise(T, Tref, tT, TOL_FP32, U64) <= 1.0
    ptil = np.concatenate([[1.0], p])
    Wref, tW = oracle.adjoint_apply(prob, ptil, Uo), abs_terms_W(prob, ptil, Uo)
    assert normwise(W, Wref, tW) <= TOL_FP32
    assert entrywise(W, Wref, tW, TOL_FP32, U32) <= 1.0


def nuclear_norm(A, B):
    """||A B^T||_* from QR factors of the thin A and B and an r x r SVD."""
    _, ra = np.linalg.qr(A)
    _, rb = np.linalg.qr(B)
    return float(np.linalg.svd(ra @ rb.T, compute_uv=False).sum())


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED], ids=["fp64", "fp32_mixed"])
def test_fullsize_mc_solve_certificate(prec):
    import scipy.sparse.linalg as sla
    d = dev()
    prob = _instance("mc_1e5x1e5_r3")
    print(f"[fullsize] mc solve: n={prob.n} m={prob.m} prec={prec}", flush=True)
    h = H.hallar_create(prob, prec, H.options(eps=1e-5, rank_cap=16))
    try:
        res = H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, 7), device=d))
        assert res["status"] == "ok", res
        U = torch.empty((prob.n, res["rank"]), dtype=torch.float64, device=d)
        p = torch.empty(prob.m, dtype=torch.float64, device=d)
        H.hallar_get_solution(h, U, p)
        U, p = U.cpu().numpy(), p.cpu().numpy()
    finally:
        H.hallar_destroy(h)
    T = oracle.a_tilde(prob, U)
    pval = float(T[0])
    assert abs(pval - res["pval"]) <= 1e-9 * (1.0 + abs(pval)), (pval, res["pval"])
    pinf = float(np.linalg.norm(T[1:] - prob.b)) / (1.0 + float(np.abs(prob.b).sum()))
    assert pinf <= 1e-5 and abs(pinf - res["pinf"]) <= 1e-9 + 1e-6 * pinf
    assert np.linalg.norm(U) <= np.sqrt(prob.tau2) * (1 + 1e-6)  # U in B_tau
    print("[fullsize] eigsh on C + A*(p)", flush=True)
    S = oracle.adjoint_sparse(prob, np.concatenate([[1.0], p]))
    lam = float(sla.eigsh(S, k=1, which="SA", tol=1e-9, return_eigenvectors=False)[0])
    theta = max(-lam, 0.0)
    # a Ritz value bounds lambda_min from above, so the solver's theta cannot
    # exceed the exact one (up to eigsh's own tolerance)
    assert res["theta"] <= theta + 1e-8 * (1.0 + theta), (res["theta"], theta)
    dval = float(-prob.b @ p - prob.tau2 * theta)
    assert abs(float(-prob.b @ p - prob.tau2 * res["theta"]) - res["dval"]) <= 1e-9 * (1.0 + abs(dval))
    gap = abs(pval - dval) / (1.0 + abs(pval) + abs(dval))
    print(f"[fullsize] theta {res['theta']:.10g} exact {theta:.10g}; gap {res['gap']:.3e} exact {gap:.3e}", flush=True)
    assert gap <= 1e-5 * (1.0 + 1e-6), (gap, pval, dval, theta, res["theta"])
    # exact recovery (Section 5.2, eq. matcomp-sdp): noise-free with
    # m = 20 r (n1 + n2) observed entries the SDP's optimum is ||A B^T||_*
    nuc = nuclear_norm(prob.meta["A"], prob.meta["B"])
    print(f"[fullsize] pval {pval:.6f} nuclear norm {nuc:.6f} rel {(pval - nuc) / (1 + nuc):.3e}", flush=True)
    assert abs(pval - nuc) <= 1e-5 * (1.0 + nuc), (pval, nuc)
