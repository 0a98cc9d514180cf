"""Pins for the oracle operators (CPU only).

* A~(UU^T) and A~*(p~)U against the dense definitions (Section 1, eq.
  Definition of Linear Operators; Section 4, eq. A tilde operator) on tiny
  random HSLR instances with duplicated triples, shared pairs, multi-entry
  constraints, diagonal entries and low-rank terms.
* The adjoint identity <A~(UU^T), p~> = <A~*(p~) U, U> (A* is the adjoint of A).
* Central finite differences of g(U) = L_beta(UU^T; p) (eq. AL function)
  against the closed-form U-gradient (eq. Grad U Space).
"""
import numpy as np
import pytest

import oracle
import sdp_instances as si
from dense_ref import dense_a_tilde, dense_adjoint


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_a_tilde_matches_dense(seed):
    prob = si.random_hslr(11, 7, seed, lowrank_nonobjective=True)
    U = np.random.default_rng(100 + seed).standard_normal((prob.n, 3))
    T = oracle.a_tilde(prob, U)
    Td = dense_a_tilde(prob, U)
    assert T.shape == (prob.m + 1,)
    np.testing.assert_allclose(T, Td, rtol=1e-12, atol=1e-12 * np.abs(Td).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adjoint_matches_dense(seed):
    prob = si.random_hslr(13, 9, seed, lowrank_nonobjective=True)
    rng = np.random.default_rng(200 + seed)
    U = rng.standard_normal((prob.n, 4))
    pt = np.concatenate([[1.0], rng.standard_normal(prob.m)])
    W = oracle.adjoint_apply(prob, pt, U)
    Wd = dense_adjoint(prob, pt, U)
    np.testing.assert_allclose(W, Wd, rtol=1e-12, atol=1e-12 * np.abs(Wd).max())


def test_objective_only_and_constraint_only_parts():
    """A~ row 0 is C . X only; rows 1..m never see C (a planted swap of the
    objective index would fail here)."""
    prob = si.random_hslr(10, 5, 7)
    U = np.random.default_rng(3).standard_normal((prob.n, 2))
    T = oracle.a_tilde(prob, U)
    prob_noC = si.Problem(prob.name, prob.n, prob.m, prob.tau2,
                          prob.row[prob.con > 0], prob.col[prob.con > 0],
                          prob.con[prob.con > 0], prob.val[prob.con > 0], prob.b)
    T2 = oracle.a_tilde(prob_noC, U)
    assert T2[0] == 0.0
    np.testing.assert_allclose(T2[1:], T[1:], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("maker", ["torus", "theta", "mc", "random"])
def test_adjoint_identity(maker):
    rng = np.random.default_rng(5)
    if maker == "torus":
        prob = si.maxcut_torus(20, 30, seed=1)
    elif maker == "theta":
        prob = si.theta_er(400, 6.0, seed=2)
    elif maker == "mc":
        prob = si.mc_planted(30, 50, 2, 700, seed=3)
    else:
        prob = si.random_hslr(200, 80, 4)
    U = rng.standard_normal((prob.n, 5))
    pt = np.concatenate([[1.0], rng.standard_normal(prob.m)])
    T = oracle.a_tilde(prob, U)
    W = oracle.adjoint_apply(prob, pt, U)
    lhs = float(T @ pt)
    rhs = float(np.sum(W * U))
    scale = float(np.abs(T * pt).sum()) + float(np.abs(W * U).sum())
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("maker", ["maxcut", "theta", "random"])
def test_gradient_finite_differences(maker):
    rng = np.random.default_rng(11)
    if maker == "maxcut":
        prob = si.maxcut_er_800(1)
        prob = si.maxcut_problem(60, *si.er_edges(60, 0.2, rng))
    elif maker == "theta":
        prob = si.theta_problem(40, *si.er_edges(40, 0.2, rng))
    else:
        prob = si.random_hslr(30, 12, 9)
    U = rng.standard_normal((prob.n, 3))
    p = rng.standard_normal(prob.m)
    beta = 3.7
    G = oracle.al_grad(prob, U, p, beta)
    for _ in range(3):
        E = rng.standard_normal(U.shape)
        h = 1e-5
        fp, _ = oracle.al_value(prob, U + h * E, p, beta)
        fm, _ = oracle.al_value(prob, U - h * E, p, beta)
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * (1.0 + abs(an))


def test_al_value_definition():
    """g = T_0 + p^T r + beta/2 ||r||^2 with r = A(UU^T) - b, checked on a
    case where every term is known by hand: one vertex, X = u^2."""
    prob = si.Problem("one", 1, 1, 4.0, row=[0, 0], col=[0, 0], con=[0, 1], val=[2.0, 1.0], b=[3.0])
    U = np.array([[1.5]])
    g, T = oracle.al_value(prob, U, np.array([0.5]), 2.0)
    assert T[0] == pytest.approx(2.0 * 2.25) and T[1] == pytest.approx(2.25)
    assert g == pytest.approx(4.5 + 0.5 * (2.25 - 3.0) + 1.0 * (2.25 - 3.0) ** 2)
