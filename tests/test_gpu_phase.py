"""Complex phase retrieval from coded diffraction patterns on the GPU
(Section 5.4, eq. phase retrieval SDP), on the real form of the Hermitian
variable (n = 2 n_c; a real column of U is u = z[:n_c] + i z[n_c:]).

* Operators against the FP64 oracle entry by entry, with error scales of a
  normwise-accurate FFT (gpu_util.cdp_terms): smooth, odd and prime lengths
  (rocFFT's Bluestein path), one to twelve patterns, r in {1, 3, 8}, both
  precisions; the adjoint identity with both sides from the GPU.
* lambda_min of C + A*(p) against LAPACK on the complex Hermitian matrix
  I + sum y a a^H (the real form doubles every eigenvalue).
* Solves: exact recovery fixes the optimum at ||x||^2 and X = x x^H; the
  primal side is recomputed by the oracle from the returned U.
* Batched with a MaxCut instance: bit-identical to solving alone.
"""
import numpy as np
import pytest

import oracle
import sdp_instances as si
from gpu_util import U32, U64, cdp_terms, dev, entrywise, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu

TOL = 1e-12
UNIT = {H.FP64: U64, H.FP32_MIXED: U32}


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED])
@pytest.mark.parametrize("nc,L,r", [(1000, 12, 3), (997, 3, 1), (4096, 2, 8), (30, 1, 5)])
def test_cdp_operators(prec, nc, L, r):
    d = dev()
    dt = torch.float64 if prec == H.FP64 else torch.float32
    prob = si.phase_retrieval_cdp(nc, L, seed=nc + L)
    print(f"[phase] operators nc={nc} L={L} r={r} prec={prec}", flush=True)
    rng = np.random.default_rng(r)
    h = H.hallar_create(prob, prec)
    try:
        Ud = torch.tensor(rng.standard_normal((prob.n, r)), dtype=dt, device=d)
        Uo = Ud.double().cpu().numpy()
        T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
        H.hallar_eval_AUUt(h, Ud, T)
        p = rng.standard_normal(prob.m)
        ptil = np.concatenate([[1.0], p])
        W = torch.empty_like(Ud)
        H.hallar_adjoint_spmm(h, torch.tensor(p, device=d), Ud, W)
        torch.cuda.synchronize()
        T, W = T.cpu().numpy(), W.double().cpu().numpy()
    finally:
        H.hallar_destroy(h)
    tT, tW = cdp_terms(prob, Uo, ptil)
    Tref = oracle.a_tilde(prob, Uo)
    assert entrywise(T, Tref, tT, TOL, U64) <= 1.0
    Wref = oracle.adjoint_apply(prob, ptil, Uo)
    assert entrywise(W, Wref, tW, TOL, UNIT[prec]) <= 1.0
    # adjoint identity with both sides from the GPU: <T, p~> = <W, U>
    lhs, rhs = float(T @ ptil), float((W * Uo).sum())
    assert abs(lhs - rhs) <= 1e-10 * (float(np.abs(tT) @ np.abs(ptil)) + float((tW * np.abs(Uo)).sum())) + \
        8 * UNIT[prec] * float(np.abs(Wref * Uo).sum())


def test_cdp_min_eig():
    d = dev()
    nc, L = 64, 4
    prob = si.phase_retrieval_cdp(nc, L, seed=3)
    y = np.random.default_rng(7).standard_normal(prob.m)
    F = np.fft.fft(np.eye(nc), axis=0, norm="ortho")          # F[k, j]
    Hm = np.eye(nc, dtype=complex)
    for l in range(L):
        A = F * prob.cdp_masks[l][None, :]                    # rows: a_{l,k}^H
        Hm += A.conj().T @ (y[l * nc:(l + 1) * nc, None] * A)
    lam_ref = float(np.linalg.eigvalsh(Hm)[0])
    h = H.hallar_create(prob, H.FP64)
    try:
        v = torch.empty(prob.n, dtype=torch.float64, device=d)
        lam, info = H.hallar_min_eig(h, torch.tensor(y, device=d), v, tol=1e-11, max_iter=5000)
        assert info["converged"]
        vv = v.cpu().numpy()
    finally:
        H.hallar_destroy(h)
    assert abs(lam - lam_ref) <= 1e-9 * max(1.0, abs(lam_ref)), (lam, lam_ref)
    G = oracle.adjoint_apply(prob, np.concatenate([[1.0], y]), np.eye(prob.n))
    assert np.linalg.norm(G @ vv - lam * vv) <= 1e-7 * max(1.0, abs(lam))


def _solve(prob, prec, eps, seed=7):
    d = dev()
    h = H.hallar_create(prob, prec, H.options(eps=eps))
    try:
        res = H.hallar_solve(h, torch.tensor(si.gaussian_u0(prob.n, seed), device=d))
        U = torch.empty((prob.n, max(res["rank"], 1)), dtype=torch.float64, device=d)
        H.hallar_get_solution(h, U, None)
        return res, U.cpu().numpy()
    finally:
        H.hallar_destroy(h)


@pytest.mark.parametrize("prec,nc", [(H.FP64, 64), (H.FP64, 1000), (H.FP32_MIXED, 1000)])
def test_cdp_exact_recovery(prec, nc):
    prob = si.phase_retrieval_cdp(nc, 12, seed=1)
    x = prob.meta["x"]
    opt = prob.tau2
    print(f"[phase] solve nc={nc} prec={prec}", flush=True)
    res, U = _solve(prob, prec, 1e-5)
    assert res["status"] == "ok", res
    assert max(res["pinf"], res["gap"], res["dinf"]) <= 1e-5
    assert abs(res["pval"] - opt) <= 1e-5 * (1 + opt), (res["pval"], opt)
    T = oracle.a_tilde(prob, U)
    assert abs(T[0] - res["pval"]) <= 1e-9 * (1 + opt)
    assert np.linalg.norm(T[1:] - prob.b) / (1 + np.abs(prob.b).sum()) <= 1e-5
    Uc = U[:nc] + 1j * U[nc:]
    X = Uc @ Uc.conj().T
    assert np.linalg.norm(X - np.outer(x, np.conj(x))) <= 1e-2 * opt   # x x^H, recovered


def test_cdp_batch_equals_alone():
    d = dev()
    rng = np.random.default_rng(4)
    i, j = si.er_edges(300, 8.0 / 299, rng)
    probs = [si.phase_retrieval_cdp(200, 12, seed=2), si.maxcut_problem(300, i, j, si.pm1_weights(i.size, rng)),
             si.phase_retrieval_cdp(81, 12, seed=5)]
    keys = ("status", "pval", "dval", "pinf", "gap", "dinf", "rank", "outer_iters", "n_fista_trials")
    alone = [_solve(p, H.FP64, 1e-5, seed=3)[0] for p in probs]
    hs = [H.hallar_create(p, H.FP64, H.options(eps=1e-5)) for p in probs]
    try:
        batch = H.hallar_solve_batch(hs, [torch.tensor(si.gaussian_u0(p.n, 3), device=d) for p in probs])
    finally:
        for h in hs:
            H.hallar_destroy(h)
    for a, b in zip(alone, batch):
        assert a["status"] == "ok", a
        for k in keys:
            assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_refuses_cdp():
    d = dev()
    prob = si.phase_retrieval_cdp(50, 2, seed=1)
    h = H.hallar_create(prob, H.FP64)
    try:
        U = torch.zeros((prob.n, 2), dtype=torch.float64, device=d)
        T = torch.zeros(prob.m + 1, dtype=torch.float64, device=d)
        with pytest.raises(H.HallarError) as ei:
            H.hallar_eval_AUUt_noalloc(h, U, T)
        assert ei.value.status == 2
    finally:
        H.hallar_destroy(h)
