"""Pins for the oracle minimum eigenpair (CPU only): LAPACK eigh on small
matrices, closed-form Laplacian spectra of cycles and tori, and ARPACK
eigsh at n = 9e4 (library routines used as checks only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import sdp_instances as si


def _G(prob, y):
    return lambda v: oracle.adjoint_apply(prob, np.concatenate([[1.0], y]), v)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_min_eig_vs_eigh(seed):
    prob = si.random_hslr(150, 60, seed)
    y = np.random.default_rng(seed).standard_normal(prob.m)
    M = oracle.adjoint_apply(prob, np.concatenate([[1.0], y]), np.eye(prob.n))
    w, Q = np.linalg.eigh(M)
    lam, v, info = oracle.min_eig(_G(prob, y), prob.n, np.random.default_rng(1).standard_normal(prob.n),
                                  tol=1e-12, kmax=60)
    assert abs(lam - w[0]) <= 1e-9 * max(1, abs(w[0]))
    assert np.linalg.norm(M @ v - lam * v) <= 1e-8 * max(1, abs(lam))
    assert abs(abs(v @ Q[:, 0]) - 1.0) <= 1e-6 or w[1] - w[0] < 1e-6


def _laplacian(n, i, j):
    A = sp.coo_matrix((np.ones(i.size), (i, j)), shape=(n, n))
    A = (A + A.T).tocsr()
    return sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A


@pytest.mark.parametrize("n", [301, 1000])
def test_cycle_closed_form(n):
    """lambda_max of the cycle Laplacian is 2 - 2 cos(2 pi floor(n/2) / n)."""
    L = _laplacian(n, *si.cycle_edges(n))
    lam, v, _ = oracle.min_eig(lambda x: -(L @ x), n, np.random.default_rng(0).standard_normal(n),
                               tol=1e-11, kmax=120, max_restarts=4000)
    exact = -(2.0 - 2.0 * math.cos(2.0 * math.pi * (n // 2) / n))
    assert abs(lam - exact) <= 1e-9


def test_torus_closed_form():
    """Torus spectrum = sums of the two cycle spectra."""
    k1, k2 = 12, 17
    n = k1 * k2
    L = _laplacian(n, *si.torus_edges(k1, k2))
    lam, _, _ = oracle.min_eig(lambda x: -(L @ x), n, np.random.default_rng(0).standard_normal(n),
                               tol=1e-12, kmax=100, max_restarts=2000)
    cyc = lambda k: 2.0 - 2.0 * math.cos(2.0 * math.pi * (k // 2) / k)
    assert abs(lam + cyc(k1) + cyc(k2)) <= 1e-9


def test_large_vs_arpack():
    prob = si.maxcut_torus(300, 300, seed=3)
    y = np.random.default_rng(4).uniform(-1, 1, prob.m)
    M = oracle.adjoint_sparse(prob, np.concatenate([[1.0], y]))
    ref = spla.eigsh(M, k=1, which="SA", tol=1e-12, v0=np.ones(prob.n))[0][0]
    lam, v, info = oracle.min_eig(lambda x: M @ x, prob.n,
                                  np.random.default_rng(2).standard_normal(prob.n), tol=1e-10, kmax=100)
    assert abs(lam - ref) <= 1e-7 * max(1.0, abs(ref))
