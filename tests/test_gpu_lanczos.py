"""GPU parity of hallar_min_eig (thick-restart Lanczos, FP64) against LAPACK
eigh on small matrices, the closed-form cycle spectrum and ARPACK eigsh at
n = 9e4 (library routines used as checks only), with the residual
||G v - lambda v|| recomputed by the oracle."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import sdp_instances as si
from gpu_util import dev, torch
from paper_2505_13719_amd import hallar as H

pytestmark = pytest.mark.gpu


def _run(prob, p, tol, v0=None, prec=H.FP64, max_iter=20000):
    d = dev()
    h = H.hallar_create(prob, prec)
    try:
        pd = torch.tensor(p, dtype=torch.float64, device=d)
        v = torch.empty(prob.n, dtype=torch.float64, device=d)
        v0d = None if v0 is None else torch.tensor(v0, dtype=torch.float64, device=d)
        lam, info = H.hallar_min_eig(h, pd, v, v0=v0d, tol=tol, max_iter=max_iter)
        return lam, v.cpu().numpy(), info
    finally:
        H.hallar_destroy(h)


@pytest.mark.parametrize("maker", ["random", "theta_lr"])
def test_min_eig_vs_eigh(maker):
    rng = np.random.default_rng(3)
    if maker == "random":
        prob = si.random_hslr(600, 250, 5, nnz=6000)
    else:
        prob = si.theta_er(700, 7.0, seed=6)
    p = rng.standard_normal(prob.m)
    ptil = np.concatenate([[1.0], p])
    M = oracle.adjoint_apply(prob, ptil, np.eye(prob.n))
    w = np.linalg.eigvalsh(M)
    lam, v, info = _run(prob, p, 1e-11)
    assert info["converged"]
    assert abs(lam - w[0]) <= 1e-9 * max(1.0, abs(w[0]))
    assert abs(np.linalg.norm(v) - 1.0) < 1e-10
    res = np.linalg.norm(oracle.adjoint_apply(prob, ptil, v) - lam * v)
    assert res <= 1e-8 * max(1.0, abs(lam))


def test_cycle_closed_form():
    """MaxCut C of a 2001-cycle with p = 0: lambda_min(-L/4) = -(2 + 2 cos(pi/n))/4."""
    n = 2001
    prob = si.maxcut_problem(n, *si.cycle_edges(n))
    lam, v, info = _run(prob, np.zeros(n), 1e-12, max_iter=200000)
    exact = -(2.0 + 2.0 * math.cos(math.pi / n)) / 4.0
    assert abs(lam - exact) <= 1e-9


def test_large_vs_arpack():
    prob = si.maxcut_torus(300, 300, seed=3)
    p = np.random.default_rng(4).uniform(-1, 1, prob.m)
    M = oracle.adjoint_sparse(prob, np.concatenate([[1.0], p]))
    ref = spla.eigsh(M, k=1, which="SA", tol=1e-12, v0=np.ones(prob.n))[0][0]
    lam, v, info = _run(prob, p, 1e-9, max_iter=100000)
    assert abs(lam - ref) <= 1e-7 * max(1.0, abs(ref))


def test_warm_start_vector():
    """An exact eigenvector as v0 converges immediately to its eigenvalue."""
    prob = si.random_hslr(300, 100, 8)
    p = np.random.default_rng(2).standard_normal(prob.m)
    ptil = np.concatenate([[1.0], p])
    M = oracle.adjoint_apply(prob, ptil, np.eye(prob.n))
    w, Q = np.linalg.eigh(M)
    lam, v, info = _run(prob, p, 1e-10, v0=Q[:, 0])
    assert abs(lam - w[0]) <= 1e-9 * max(1, abs(w[0]))
    assert info["iters"] <= 16
