"""Oracle minimum eigenpair (FP64) — test infrastructure only.

Alg. 1 step ii of the cuHALLaR paper needs (lambda_min(G), v_min(G)) of
G = C + A*(p + beta (A(YY^T) - b)) but does not name an eigensolver.  This is
the textbook symmetric Lanczos process with full reorthogonalisation (two
classical Gram-Schmidt passes per step), Rayleigh-Ritz on the tridiagonal
T_k = V_k^T G V_k, and explicit restart from the best Ritz vector when the
basis reaches kmax vectors.  Convergence: the Ritz residual
||G x - theta x|| = beta_k |s_k| <= max(atol, tol * max(1, |theta|)).
The smallest Ritz value is within that residual of an eigenvalue of G.
"""
from __future__ import annotations

import numpy as np


def min_eig(matvec, n, v0, tol=1e-10, kmax=80, max_restarts=400, atol=0.0):
    """Returns (lam, v, info) with info = dict(iters, residual, restarts).
    Stops when the Ritz residual is <= max(atol, tol * max(1, |theta|))."""
    v = np.asarray(v0, np.float64).copy()
    nv = np.linalg.norm(v)
    if nv == 0.0:
        v = np.ones(n)
        nv = np.sqrt(n)
    v /= nv
    kmax = max(2, min(kmax, n))
    iters = 0
    lam, x, res = None, v, np.inf
    for restart in range(max_restarts):
        V = np.zeros((kmax + 1, n))
        V[0] = v
        alpha = np.zeros(kmax)
        beta = np.zeros(kmax)
        k = 0
        breakdown = False
        for j in range(kmax):
            w = matvec(V[j])
            iters += 1
            alpha[j] = V[j] @ w
            for _ in range(2):                       # CGS2 full reorthogonalisation
                w = w - V[: j + 1].T @ (V[: j + 1] @ w)
            beta[j] = np.linalg.norm(w)
            k = j + 1
            if beta[j] <= 1e-14 * max(1.0, abs(alpha[j])):
                breakdown = True                     # invariant subspace: Ritz values exact
                break
            V[j + 1] = w / beta[j]
        Tk = np.diag(alpha[:k]) + np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
        theta, S = np.linalg.eigh(Tk)
        lam = float(theta[0])
        s = S[:, 0]
        x = V[:k].T @ s
        x /= np.linalg.norm(x)
        res = 0.0 if breakdown else float(beta[k - 1] * abs(s[-1]))
        if res <= max(atol, tol * max(1.0, abs(lam))) or k == n:
            break
        v = x
    return lam, x, {"iters": iters, "residual": res, "restarts": restart}
