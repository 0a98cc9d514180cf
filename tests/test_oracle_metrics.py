"""Pins for the oracle's stopping quantities (CPU only).

`oracle.metrics` computes the three relative errors of eq. termination2
(Section 5.1): primal infeasibility ||A(X) - b||_2 / (1 + ||b||_1), the
relative duality gap |pval - dval| / (1 + |pval| + |dval|) and the dual
infeasibility max(0, -lambda_min(S)) / (1 + ||C||_1).  `oracle.c_l1_norm`
is the ||C||_1 of that formula, read as the entrywise l1 norm of the full
symmetric C with its low-rank part included.

The expected numbers below were worked out by hand from those definitions
(the arithmetic is written next to each), so a swapped norm, a dropped
"1 +", a missing symmetric twin of an off-diagonal entry or a lost low-rank
term fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
import sdp_instances as si


def test_metrics_worked_example():
    # triangle K3 MaxCut: b = (1, 1, 1), ||b||_1 = 3, ||b||_2 = sqrt(3)
    i, j = si.complete_edges(3)
    prob = si.maxcut_problem(3, i, j)
    # T = (C.X, X_11, X_22, X_33) = (-1.25, 1.5, 1.0, 0.5): r = (0.5, 0, -0.5)
    T = np.array([-1.25, 1.5, 1.0, 0.5])
    pinf, gap, dinf = oracle.metrics(prob, pval=-2.0, dval=-2.5, T_Y=T, lam_min_S=-0.3, cnorm1=2.0)
    # pinf = sqrt(0.25 + 0.25) / (1 + 3) = 0.70710678... / 4
    assert pinf == pytest.approx(0.1767766952966369, rel=1e-14)
    # gap = |-2 + 2.5| / (1 + 2 + 2.5) = 0.5 / 5.5
    assert gap == pytest.approx(0.09090909090909091, rel=1e-14)
    # dinf = 0.3 / (1 + 2)
    assert dinf == pytest.approx(0.1, rel=1e-14)


def test_metrics_signs_and_clamps():
    i, j = si.complete_edges(3)
    prob = si.maxcut_problem(3, i, j)
    T = np.array([0.0, 1.0, 1.0, 1.0])                 # feasible: r = 0
    pinf, gap, dinf = oracle.metrics(prob, pval=3.0, dval=-1.0, T_Y=T, lam_min_S=0.25, cnorm1=5.0)
    assert pinf == 0.0
    # gap = |3 - (-1)| / (1 + 3 + 1) = 4 / 5: absolute values of both objectives
    assert gap == pytest.approx(0.8, rel=1e-14)
    # lambda_min(S) >= 0: no dual infeasibility
    assert dinf == 0.0


def test_metrics_b_with_mixed_signs():
    # theta-like data with b = 0 except a mixed-sign pair of constraints:
    # ||b||_1 = 2 + 3 = 5 (an l2 norm would give sqrt(13))
    i, j = si.cycle_edges(4)
    prob = si.theta_problem(4, i, j)
    prob.b = np.array([2.0, -3.0, 0.0, 0.0])
    T = np.array([-4.0, 2.0, -1.0, 4.0, 0.0])          # r = (0, 2, 4, 0), ||r||_2 = sqrt(20)
    pinf, _, _ = oracle.metrics(prob, pval=0.0, dval=0.0, T_Y=T, lam_min_S=0.0, cnorm1=0.0)
    assert pinf == pytest.approx(math.sqrt(20.0) / 6.0, rel=1e-14)


def test_c_l1_norm_sparse_maxcut_triangle():
    # C = -L/4 of K3: diagonal -2/4 (three entries), off-diagonal +1/4 (six
    # entries of the full symmetric matrix): 3 * 0.5 + 6 * 0.25 = 3.0
    i, j = si.complete_edges(3)
    assert oracle.c_l1_norm(si.maxcut_problem(3, i, j)) == pytest.approx(3.0, rel=1e-15)


def test_c_l1_norm_signed_weights():
    # path 0-1-2 with weights +1 and -1: degrees (1, 0, -1), L = [[1,-1,0],[-1,0,1],[0,1,-1]]
    # C = -L/4: |diag| = 0.25 + 0 + 0.25, off-diagonal 4 entries of 0.25: total 1.5
    prob = si.maxcut_problem(3, np.array([0, 1]), np.array([1, 2]), np.array([1.0, -1.0]))
    assert oracle.c_l1_norm(prob) == pytest.approx(1.5, rel=1e-15)


@pytest.mark.parametrize("n", [5, 40])
def test_c_l1_norm_theta_dense_lowrank(n):
    # C = -e e^T: every one of the n^2 entries has |C_ij| = 1 (dense branch, n <= 4096)
    i, j = si.cycle_edges(n)
    assert oracle.c_l1_norm(si.theta_problem(n, i, j)) == pytest.approx(float(n * n), rel=1e-15)


def test_c_l1_norm_theta_large_n():
    # n > 4096 takes the closed form |D| n^2 of the all-ones K (n = 5000: 2.5e7)
    n = 5000
    i, j = si.cycle_edges(n)
    assert oracle.c_l1_norm(si.theta_problem(n, i, j)) == pytest.approx(25_000_000.0, rel=1e-15)


def test_c_l1_norm_sparse_plus_lowrank():
    # C = [[1, 2], [2, 0]] (sparse: C_00 = 1, C_01 = 2) plus K D K^T with
    # K = (1, -1)^T, D = [[3]]: K D K^T = [[3, -3], [-3, 3]].
    # Full C = [[4, -1], [-1, 3]]: l1 = 4 + 1 + 1 + 3 = 9 (entries cancel
    # inside the sum, so adding the two norms, 5 + 12 = 17, would be wrong)
    prob = si.Problem(name="c2x2", n=2, m=1, tau2=2.0,
                      row=np.array([0, 0, 1]), col=np.array([0, 1, 1]), con=np.array([0, 0, 1]),
                      val=np.array([1.0, 2.0, 1.0]), b=np.array([1.0]),
                      lr_con=[0], lr_K=[np.array([[1.0], [-1.0]])], lr_D=[np.array([[3.0]])])
    assert oracle.c_l1_norm(prob) == pytest.approx(9.0, rel=1e-15)


def test_c_l1_norm_ignores_constraints():
    # entries of A_1..A_m (con > 0) are not part of C: MC data C = I/2 only
    prob = si.mc_planted(4, 5, 1, 12, seed=0)
    assert oracle.c_l1_norm(prob) == pytest.approx(4.5, rel=1e-15)   # 9 diagonal entries of 1/2
