"""hallar_eval_AUUt_noalloc (the allocation-free evaluation, for callers that
cannot allocate at call time) against hallar_eval_AUUt through the C ABI.

Both run the same kernels in the same order on the same tiles, so T must be
bit-identical.  Two calls in a row share the GPU's scratch array, the second
with a smaller input (fewer columns, then a smaller instance), in direct and
general constraint modes, with U read in place and packed, with and without
a low-rank objective term.  An instance whose scratch need exceeds the
array is rejected with E_INVALID.
"""
import numpy as np
import pytest

import oracle
import sdp_instances as si
from gpu_util import abs_terms_T, dev, normwise, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu


def _pair(h, prob, U):
    d = dev()
    T1 = torch.full((prob.m + 1,), float("nan"), dtype=torch.float64, device=d)
    T2 = torch.full_like(T1, float("nan"))
    H.hallar_eval_AUUt_noalloc(h, U, T1)
    H.hallar_eval_AUUt(h, U, T2)
    torch.cuda.synchronize()
    return T1.cpu(), T2.cpu()


CASES = [
    ("mc_fp32", lambda: si.mc_planted(600, 800, 3, 50000, seed=3), H.FP32_MIXED),
    ("theta_lowrank_fp64", lambda: si.theta_er(3000, 8.0, seed=2), H.FP64),
    ("general_fp64", lambda: si.random_hslr(1200, 500, 1, nnz=15000), H.FP64),
    ("torus_fp32", lambda: si.maxcut_torus(70, 90, seed=1), H.FP32_MIXED),
]


@pytest.mark.parametrize("name,maker,prec", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_eval(name, maker, prec):
    d = dev()
    dt = torch.float64 if prec == H.FP64 else torch.float32
    big = maker()
    small = si.maxcut_er_800(1) if prec == H.FP64 else si.mc_planted(200, 300, 2, 8000, seed=4)
    rng = np.random.default_rng(5)
    hb = H.hallar_create(big, prec)
    hs = H.hallar_create(small, prec)
    try:
        # first call: 8 columns (in place: a column bucket in both precisions)
        U8 = torch.tensor(rng.standard_normal((big.n, 8)), dtype=dt, device=d)
        a, b = _pair(hb, big, U8)
        assert torch.equal(a, b)
        Uo = U8.double().cpu().numpy()
        assert normwise(a.numpy(), oracle.a_tilde(big, Uo), abs_terms_T(big, Uo)) <= 1e-5
        # second call, same handle, fewer columns: packed through the scratch
        U3 = torch.tensor(rng.standard_normal((big.n, 3)), dtype=dt, device=d)
        a, b = _pair(hb, big, U3)
        assert torch.equal(a, b)
        # then a smaller instance on another handle
        Us = torch.tensor(rng.standard_normal((small.n, 2)), dtype=dt, device=d)
        a, b = _pair(hs, small, Us)
        assert torch.equal(a, b)
        # the handle's own evaluation is unaffected by the scratch calls
        a2, b2 = _pair(hb, big, U3)
        assert torch.equal(a2, b2)
    finally:
        H.hallar_destroy(hb)
        H.hallar_destroy(hs)


def test_noalloc_rejects_oversized_scratch():
    """FP64, r = 31 on 302,500 vertices: the packed U alone (n x 32 doubles,
    77 MB) exceeds the 64 MiB array; the call is refused, nothing runs."""
    d = dev()
    prob = si.maxcut_torus(550, 550, seed=1)
    h = H.hallar_create(prob, H.FP64)
    try:
        U = torch.zeros((prob.n, 31), dtype=torch.float64, device=d)
        T = torch.zeros(prob.m + 1, dtype=torch.float64, device=d)
        with pytest.raises(H.HallarError) as ei:
            H.hallar_eval_AUUt_noalloc(h, U, T)
        assert ei.value.status == 1
        assert float(T.abs().max()) == 0.0
    finally:
        H.hallar_destroy(h)
