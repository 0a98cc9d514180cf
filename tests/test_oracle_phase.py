"""Pins for the oracle's coded-diffraction operators (Section 5.4, eq.
phase retrieval SDP) on the real form of the complex Hermitian variable.

* Brute force: the measurement vectors a_{l,k} written out from the DFT's
  definition (a matrix of exp(-2 pi i jk/n)/sqrt(n) built entry by entry, no
  FFT) and the real 2n x 2n matrices [[Re H, -Im H], [Im H, Re H]] of
  H = a a^H: A~(ZZ^T) and A~*(p~)Z against them on tiny instances.
* Closed form: sum_{l,k} a a^H = diag(sum_l |d_l|^2) (F unitary), so
  A*(1) Z multiplies each row by that diagonal.
* The real form's spectrum is the complex matrix's, each eigenvalue twice:
  the oracle's Lanczos lambda_min against LAPACK on the complex Hermitian
  I + sum y a a^H.
* Exact recovery (the SDP's solution is x x^H, value ||x||^2): oracle
  solves reach it, and the complex X they return is x x^H.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import sdp_instances as si


def _dft(n):
    F = np.empty((n, n), complex)
    for k in range(n):
        for j in range(n):
            F[k, j] = cmath.exp(-2j * math.pi * j * k / n) / math.sqrt(n)
    return F


def _real_form(H):
    return np.block([[H.real, -H.imag], [H.imag, H.real]])


def _dense_constraints(prob):
    """The real 2n x 2n matrix of every constraint, from the definition."""
    L, nc = prob.cdp_masks.shape
    F = _dft(nc)
    mats = []
    for l in range(L):
        for k in range(nc):
            a = np.conj(F[k] * prob.cdp_masks[l])        # a^H u = sum_j F_kj d_lj u_j
            mats.append(_real_form(np.outer(a, np.conj(a))))
    return mats


@pytest.mark.parametrize("nc,L", [(5, 3), (6, 2)])
def test_operators_brute_force(nc, L):
    prob = si.phase_retrieval_cdp(nc, L, seed=nc)
    mats = _dense_constraints(prob)
    rng = np.random.default_rng(1)
    Z = rng.standard_normal((prob.n, 3))
    X = Z @ Z.T
    T = oracle.a_tilde(prob, Z)
    assert abs(T[0] - np.trace(X)) <= 1e-13 * np.trace(X)
    ref = np.array([np.sum(A * X) for A in mats])
    assert np.abs(T[1:] - ref).max() <= 1e-13 * (1 + np.abs(ref).max())
    pt = rng.standard_normal(prob.m + 1)
    G = pt[0] * np.eye(prob.n) + sum(p * A for p, A in zip(pt[1:], mats))
    W = oracle.adjoint_apply(prob, pt, Z)
    assert np.abs(W - G @ Z).max() <= 1e-13 * (1 + np.abs(G @ Z).max())


def test_adjoint_of_ones_closed_form():
    prob = si.phase_retrieval_cdp(24, 4, seed=2)
    Z = np.random.default_rng(3).standard_normal((prob.n, 2))
    pt = np.concatenate([[0.0], np.ones(prob.m)])
    dsum = (np.abs(prob.cdp_masks) ** 2).sum(axis=0)
    W = oracle.adjoint_apply(prob, pt, Z)
    ref = np.concatenate([dsum, dsum])[:, None] * Z
    assert np.abs(W - ref).max() <= 1e-13 * np.abs(ref).max()


def test_measurements_and_phase_invariance():
    prob = si.phase_retrieval_cdp(20, 12, seed=4)
    x = prob.meta["x"]
    for phi in (0.0, 0.7, 2.0):
        y = cmath.exp(1j * phi) * x
        T = oracle.a_tilde(prob, np.concatenate([y.real, y.imag])[:, None])
        assert abs(T[0] - prob.tau2) <= 1e-12 * prob.tau2
        assert np.abs(T[1:] - prob.b).max() <= 1e-12 * np.abs(prob.b).max()


def test_real_form_spectrum():
    prob = si.phase_retrieval_cdp(16, 3, seed=5)
    L, nc = prob.cdp_masks.shape
    F = _dft(nc)
    y = np.random.default_rng(6).standard_normal(prob.m)
    H = np.eye(nc, dtype=complex)
    for l in range(L):
        for k in range(nc):
            a = np.conj(F[k] * prob.cdp_masks[l])
            H += y[l * nc + k] * np.outer(a, np.conj(a))
    lam_c = np.linalg.eigvalsh(H)
    lam_r = np.linalg.eigvalsh(oracle.adjoint_apply(prob, np.concatenate([[1.0], y]), np.eye(prob.n)))
    assert np.abs(np.sort(np.repeat(lam_c, 2)) - lam_r).max() <= 1e-12 * (1 + np.abs(lam_c).max())
    lam, v, _ = oracle.min_eig(lambda u: oracle.adjoint_apply(prob, np.concatenate([[1.0], y]), u), prob.n,
                               tol=1e-11, v0=np.random.default_rng(1).standard_normal(prob.n))
    assert abs(lam - lam_c[0]) <= 1e-9 * (1 + abs(lam_c[0]))


@pytest.mark.parametrize("nc", [16, 48])
def test_exact_recovery(nc):
    prob = si.phase_retrieval_cdp(nc, 12, seed=1)
    x = prob.meta["x"]
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 7), oracle.Options(eps=1e-7))
    assert res.status == "ok"
    assert abs(res.pval - prob.tau2) <= 1e-6 * (1 + prob.tau2), (res.pval, prob.tau2)
    Uc = res.U[:nc] + 1j * res.U[nc:]
    X = Uc @ Uc.conj().T
    assert np.linalg.norm(X - np.outer(x, np.conj(x))) <= 1e-4 * prob.tau2
