"""GPU parity of the operator entry points against the FP64 oracle.

hallar_eval_AUUt (A~(UU^T), Algorithms 2-3) and hallar_adjoint_spmm
(A~*(1,p)U, Algorithms 4-5) through the C ABI, in FP64 (error <= 1e-12 of
the absolute terms) and FP32-mixed (<= 1e-5), normwise and entry by entry
(each output within tol times its own absolute terms plus 4 units of
roundoff of the stored result), on instances that
span several tiles with ragged tails: general multi-entry constraints,
MaxCut on ER graphs and tori, Lovasz theta with the low-rank objective,
matrix completion; edge cases r = 1, r = 64, ldu > r, n = 1, m = 0.
"""
import numpy as np
import pytest

import oracle
import sdp_instances as si
from gpu_util import U32, U64, abs_terms_T, abs_terms_W, dev, entrywise, normwise, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu

TOL = {H.FP64: 1e-12, H.FP32_MIXED: 1e-5}
UNIT = {H.FP64: U64, H.FP32_MIXED: U32}


def _cases():
    rng = np.random.default_rng(0)
    i, j = si.er_edges(3000, 0.004, rng)
    yield "random_general", si.random_hslr(1500, 700, 1, nnz=20000)
    yield "maxcut_er", si.maxcut_problem(3000, i, j, si.pm1_weights(i.size, rng))
    yield "torus", si.maxcut_torus(97, 61, seed=1)
    yield "theta_lr", si.theta_er(4000, 9.0, seed=2)
    yield "mc", si.mc_planted(700, 900, 3, 60000, seed=3)


CASES = list(_cases())


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_MIXED])
@pytest.mark.parametrize("name,prob", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("r", [1, 3, 5, 32])
def test_eval_and_adjoint_parity(prec, name, prob, r):
    d = dev()
    dt = torch.float64 if prec == H.FP64 else torch.float32
    rng = np.random.default_rng(r)
    U = rng.standard_normal((prob.n, r))
    p = rng.standard_normal(prob.m)
    h = H.hallar_create(prob, prec)
    try:
        Ud = torch.tensor(U, dtype=dt, device=d)
        T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
        H.hallar_eval_AUUt(h, Ud, T)
        Uo = Ud.double().cpu().numpy()       # the exact values the GPU multiplied
        Tref = oracle.a_tilde(prob, Uo)
        tT = abs_terms_T(prob, Uo)
        assert normwise(T.cpu().numpy(), Tref, tT) <= TOL[prec]
        assert entrywise(T.cpu().numpy(), Tref, tT, TOL[prec], U64) <= 1.0
        pd = torch.tensor(p, dtype=torch.float64, device=d)
        W = torch.empty((prob.n, r), dtype=dt, device=d)
        H.hallar_adjoint_spmm(h, pd, Ud, W)
        ptil = np.concatenate([[1.0], p])
        Wref = oracle.adjoint_apply(prob, ptil, Uo)
        tW = abs_terms_W(prob, ptil, Uo)
        assert normwise(W.double().cpu().numpy(), Wref, tW) <= TOL[prec]
        assert entrywise(W.double().cpu().numpy(), Wref, tW, TOL[prec], UNIT[prec]) <= 1.0
    finally:
        H.hallar_destroy(h)


def test_strided_and_wide_inputs():
    """ldu > r and r = 64 (the widest bucket) in FP64."""
    d = dev()
    prob = si.maxcut_torus(40, 37, seed=4)
    rng = np.random.default_rng(7)
    h = H.hallar_create(prob, H.FP64)
    try:
        for r, ld in ((64, 64), (3, 11)):
            big = torch.tensor(rng.standard_normal((prob.n, ld)), dtype=torch.float64, device=d)
            Ud = big[:, :r]
            T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
            H.hallar_eval_AUUt(h, Ud, T)
            Uo = Ud.cpu().numpy()
            assert normwise(T.cpu().numpy(), oracle.a_tilde(prob, Uo), abs_terms_T(prob, Uo)) <= 1e-12
            p = torch.tensor(rng.standard_normal(prob.m), device=d)
            Wbig = torch.zeros((prob.n, ld + 2), dtype=torch.float64, device=d)
            W = Wbig[:, :r]
            H.hallar_adjoint_spmm(h, p, Ud, W)
            ptil = np.concatenate([[1.0], p.cpu().numpy()])
            ref = oracle.adjoint_apply(prob, ptil, Uo)
            assert normwise(W.cpu().numpy(), ref, abs_terms_W(prob, ptil, Uo)) <= 1e-12
            assert float(Wbig[:, r:].abs().max()) == 0.0      # nothing written past r
    finally:
        H.hallar_destroy(h)


def test_degenerate_sizes():
    """n = 1 (one vertex, one constraint) and m = 0 (theta of an empty graph)."""
    d = dev()
    one = si.Problem("one", 1, 1, 4.0, row=[0, 0], col=[0, 0], con=[0, 1], val=[2.0, 1.0], b=[3.0])
    e = np.zeros(0, np.int64)
    empty = si.theta_problem(7, e, e)
    for prob in (one, empty):
        h = H.hallar_create(prob, H.FP64)
        try:
            U = torch.tensor(np.random.default_rng(1).standard_normal((prob.n, 2)), device=d)
            T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
            H.hallar_eval_AUUt(h, U, T)
            np.testing.assert_allclose(T.cpu().numpy(), oracle.a_tilde(prob, U.cpu().numpy()), rtol=1e-13, atol=1e-13)
            p = torch.ones(max(prob.m, 1), dtype=torch.float64, device=d)
            W = torch.empty_like(U)
            H.hallar_adjoint_spmm(h, p, U, W)
            ref = oracle.adjoint_apply(prob, np.concatenate([[1.0], np.ones(prob.m)]), U.cpu().numpy())
            np.testing.assert_allclose(W.cpu().numpy(), ref, rtol=1e-13, atol=1e-13)
        finally:
            H.hallar_destroy(h)


def test_adjoint_identity_on_device():
    """<A~(UU^T), p~> = <A~*(p~)U, U> with both sides from the GPU."""
    d = dev()
    prob = si.theta_er(3000, 8.0, seed=9)
    rng = np.random.default_rng(3)
    h = H.hallar_create(prob, H.FP64)
    try:
        U = torch.tensor(rng.standard_normal((prob.n, 4)), device=d)
        p = rng.standard_normal(prob.m)
        T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
        H.hallar_eval_AUUt(h, U, T)
        W = torch.empty_like(U)
        H.hallar_adjoint_spmm(h, torch.tensor(p, device=d), U, W)
        lhs = float(T.cpu().numpy() @ np.concatenate([[1.0], p]))
        rhs = float((W * U).sum())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + float((W * U).abs().sum()))
    finally:
        H.hallar_destroy(h)


def test_repeatable_bitwise():
    """Fixed-order reductions: two evaluations give identical bits."""
    d = dev()
    prob = si.maxcut_torus(120, 130, seed=5)
    h = H.hallar_create(prob, H.FP32_MIXED)
    try:
        U = torch.randn(prob.n, 16, device=d, dtype=torch.float32, generator=torch.Generator(device=d).manual_seed(1))
        T1 = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
        T2 = torch.empty_like(T1)
        H.hallar_eval_AUUt(h, U, T1)
        H.hallar_eval_AUUt(h, U, T2)
        assert torch.equal(T1, T2)
    finally:
        H.hallar_destroy(h)


@pytest.mark.parametrize("prec,r", [(H.FP32_MIXED, 4), (H.FP32_MIXED, 16), (H.FP64, 2), (H.FP64, 8)])
def test_in_place_matches_packed(prec, r):
    """With r a column bucket and ld = r the entry points read U and write W
    in place; a strided view of the same values goes through the packing
    copy.  Both run the same kernels on the same rows: identical bits."""
    d = dev()
    dt = torch.float64 if prec == H.FP64 else torch.float32
    prob = si.mc_planted(500, 700, 3, 40000, seed=5)
    rng = np.random.default_rng(2)
    h = H.hallar_create(prob, prec)
    try:
        U = torch.tensor(rng.standard_normal((prob.n, r)), dtype=dt, device=d)
        big = torch.zeros((prob.n, r + 3), dtype=dt, device=d)
        big[:, :r] = U
        Us = big[:, :r]
        p = torch.tensor(rng.standard_normal(prob.m), device=d)
        out = []
        for X in (U, Us):
            T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
            H.hallar_eval_AUUt(h, X, T)
            W = torch.empty((prob.n, r), dtype=dt, device=d)
            H.hallar_adjoint_spmm(h, p, X, W)
            out.append((T.cpu(), W.cpu()))
        assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
        Uo = U.double().cpu().numpy()
        assert normwise(out[0][0].numpy(), oracle.a_tilde(prob, Uo), abs_terms_T(prob, Uo)) <= TOL[prec]
    finally:
        H.hallar_destroy(h)


def test_async_calls_keep_their_parameters():
    """Back-to-back asynchronous calls with different inputs and role tables
    (in place and packed, eval and adjoint) each see their own parameters:
    the results equal the same calls made one at a time with a sync between
    them, bit for bit; an eigen solve on the same handle afterwards runs."""
    d = dev()
    prob = si.mc_planted(700, 900, 3, 60000, seed=3)
    rng = np.random.default_rng(4)
    h = H.hallar_create(prob, H.FP64)
    try:
        U1 = torch.tensor(rng.standard_normal((prob.n, 4)), device=d)                 # in place
        U2 = torch.tensor(rng.standard_normal((prob.n, 3)), device=d)                 # packed
        U3 = torch.tensor(rng.standard_normal((prob.n, 8)), device=d)                 # in place, wider
        p = torch.tensor(rng.standard_normal(prob.m), device=d)

        def calls(sync):
            out = []
            for U in (U1, U2, U3):
                T = torch.empty(prob.m + 1, dtype=torch.float64, device=d)
                H.hallar_eval_AUUt(h, U, T)
                if sync:
                    torch.cuda.synchronize()
                W = torch.empty_like(U)
                H.hallar_adjoint_spmm(h, p, U, W)
                if sync:
                    torch.cuda.synchronize()
                out.append((T, W))
            torch.cuda.synchronize()
            return [(T.cpu(), W.cpu()) for T, W in out]

        ref = calls(True)
        got = calls(False)
        for (Tr, Wr), (Tg, Wg) in zip(ref, got):
            assert torch.equal(Tr, Tg) and torch.equal(Wr, Wg)
        v = torch.empty(prob.n, dtype=torch.float64, device=d)
        lam, info = H.hallar_min_eig(h, p * 1e-3, v, tol=1e-9, max_iter=2000)
        assert np.isfinite(lam)
    finally:
        H.hallar_destroy(h)
