"""Lovasz theta of the Hamming graphs H(d, 2) on the GPU (Section 5.3,
eq. lovasz, Table tab:reduced_hamming_graphs: the maximum stable set
experiments).  H(d, 2) joins d-bit words at Hamming distance one; it is
bipartite, hence perfect, so theta = alpha = n / 2 exactly (n = 2^d).

The solve's objective must sit within 1e-5 relative of -n/2 with relative
gap, infeasibility and dual infeasibility <= 1e-5, in FP64 up to
d = 21 (n = 2,097,152, 22,020,096 edge constraints) and in FP32-mixed; its
primal side is recomputed without the GPU from the returned U (the oracle's
A~(UU^T)), and for the sizes where scipy's eigsh finishes in seconds, the
dual value from the exact lambda_min of C + A*(p) certifies the result from
below: dval_exact <= theta bound, and the exact gap meets eps.
"""
import numpy as np
import pytest

import oracle
import sdp_instances as si
from gpu_util import dev, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu


def _solve(d, prec):
    dv = dev()
    n = 1 << d
    prob = si.theta_problem(n, *si.hypercube_edges(d))
    print(f"[hamming] d={d} n={n} m={prob.m} prec={prec}", flush=True)
    h = H.hallar_create(prob, prec, H.options(eps=1e-5))
    try:
        res = H.hallar_solve(h, torch.tensor(si.gaussian_u0(n, 7), device=dv))
        U = torch.empty((n, max(res["rank"], 1)), dtype=torch.float64, device=dv)
        p = torch.empty(prob.m, dtype=torch.float64, device=dv)
        H.hallar_get_solution(h, U, p)
        return prob, res, U.cpu().numpy(), p.cpu().numpy()
    finally:
        H.hallar_destroy(h)


@pytest.mark.parametrize("d,prec", [(10, H.FP64), (12, H.FP64), (14, H.FP64), (16, H.FP64), (18, H.FP64),
                                    (21, H.FP64), (12, H.FP32_MIXED), (16, H.FP32_MIXED), (21, H.FP32_MIXED)])
def test_theta_hamming_is_half_n(d, prec):
    prob, res, U, p = _solve(d, prec)
    n = prob.n
    assert res["status"] == "ok", res
    assert max(res["pinf"], res["gap"], res["dinf"]) <= 1e-5
    assert abs(res["pval"] + n / 2) <= 1e-5 * (1 + n / 2), (res["pval"], -n / 2)
    # primal side without the GPU
    T = oracle.a_tilde(prob, U)
    assert abs(T[0] - res["pval"]) <= 1e-9 * (1 + n / 2)
    assert np.linalg.norm(T[1:]) / (1 + np.abs(prob.b).sum()) <= 1e-5
    assert np.linalg.norm(U) <= 1 + 1e-6


@pytest.mark.parametrize("d", [12, 14])
def test_theta_hamming_certificate(d):
    """The dual value recomputed with scipy's lambda_min of C + A*(p)
    (C = -ee^T as a rank-one update of the sparse A*(p)) bounds theta = n/2
    from above up to eps, and the exact relative gap meets eps."""
    import scipy.sparse.linalg as sla
    prob, res, U, p = _solve(d, H.FP64)
    n = prob.n
    S = oracle.adjoint_sparse(prob, np.concatenate([[0.0], p]))     # A*(p), sparse
    e = np.ones(n)
    op = sla.LinearOperator((n, n), matvec=lambda v: S @ v - e * (e @ v), dtype=np.float64)
    lam = float(sla.eigsh(op, k=1, which="SA", tol=1e-10, return_eigenvectors=False)[0])
    theta = max(-lam, 0.0)
    dval = float(-prob.b @ p - prob.tau2 * theta)
    assert res["theta"] <= theta + 1e-8 * (1 + theta)
    assert dval <= -n / 2 + 1e-5 * (1 + n / 2)          # weak duality with the exact lambda_min
    gap = abs(res["pval"] - dval) / (1 + abs(res["pval"]) + abs(dval))
    assert gap <= 1e-5, gap
