"""Dense references for tiny instances (n <= ~60) used to pin the oracle.

They build every data matrix A_l as a full n x n array and apply the
definitions of Section 1 (eq. Definition of Linear Operators) and Section 4
(eq. A tilde operator) literally, with no symmetry weights, index lists or
low-rank shortcuts.  Also: brute-force MaxCut / stable-set values and a
small dense SDP solver that works directly on X (augmented Lagrangian with
exact projection onto the spectraplex), sharing nothing with the
factorised method.
"""
import itertools
import math

import numpy as np


def dense_mats(prob):
    """[A_0 = C, A_1, ..., A_m] as dense symmetric n x n arrays."""
    mats = np.zeros((prob.m + 1, prob.n, prob.n))
    for i, j, l, v in zip(prob.row, prob.col, prob.con, prob.val):
        mats[l, i, j] += v
        if i != j:
            mats[l, j, i] += v
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        mats[l] += K @ D @ K.T
    return mats


def dense_a_tilde(prob, U):
    X = U @ U.T
    return np.array([np.sum(A * X) for A in dense_mats(prob)])


def dense_adjoint(prob, ptilde, U):
    M = np.tensordot(np.asarray(ptilde), dense_mats(prob), axes=1)
    return M @ U


def brute_maxcut(n, i, j, w):
    """max over +-1 vectors x of sum_{edges} w_ij (1 - x_i x_j)/2."""
    best = -np.inf
    i = np.asarray(i); j = np.asarray(j); w = np.asarray(w, float)
    for chunk in range(0, 1 << (n - 1), 1 << 12):
        masks = np.arange(chunk, min(chunk + (1 << 12), 1 << (n - 1)))
        bits = (masks[:, None] >> np.arange(n)[None, :]) & 1
        cut = ((bits[:, i] != bits[:, j]) * w[None, :]).sum(axis=1)
        best = max(best, cut.max())
    return float(best)


def brute_stable(n, i, j):
    """Stability number alpha(G) by enumeration."""
    masks = np.arange(1 << n)
    bad = np.zeros(masks.size, bool)
    for a, b in zip(i, j):
        bad |= ((masks >> a) & 1).astype(bool) & ((masks >> b) & 1).astype(bool)
    sizes = np.array([bin(x).count("1") for x in masks])
    return int(sizes[~bad].max())


def proj_spectraplex(X, tau2):
    """Euclidean projection onto {X PSD, Tr X <= tau2}."""
    lam, Q = np.linalg.eigh(0.5 * (X + X.T))
    mu = np.maximum(lam, 0.0)
    if mu.sum() > tau2:
        s = np.sort(lam)[::-1]
        cs = np.cumsum(s)
        k = np.nonzero(s - (cs - tau2) / np.arange(1, s.size + 1) > 0)[0][-1]
        shift = (cs[k] - tau2) / (k + 1)
        mu = np.maximum(lam - shift, 0.0)
    return (Q * mu) @ Q.T


def dense_sdp(prob, tol=1e-9, max_outer=400, inner=4000):
    """min C.X s.t. A(X) = b, X in spectraplex, by an augmented Lagrangian
    on the full matrix X with accelerated projected-gradient subproblems.
    Returns (pval, dval, X, p) with dval a valid lower bound computed from
    a dense eigen decomposition."""
    mats = dense_mats(prob)
    C, As = mats[0], mats[1:]
    m, n = prob.m, prob.n
    Amat = As.reshape(m, -1)
    normA2 = np.linalg.norm(Amat, 2) ** 2 if m else 0.0
    X = np.eye(n) * prob.tau2 / n
    p = np.zeros(m)
    beta = 1.0
    pval = dval = None
    for outer in range(max_outer):
        L = max(beta * normA2, 1e-3 * np.linalg.norm(C, 2), 1e-12)
        Y, t = X.copy(), 1.0
        for _ in range(inner):
            G = C + (Amat.T @ (p + beta * (Amat @ Y.reshape(-1) - prob.b))).reshape(n, n)
            Xn = proj_spectraplex(Y - G / L, prob.tau2)
            tn = 0.5 * (1 + math.sqrt(1 + 4 * t * t))
            Y = Xn + ((t - 1) / tn) * (Xn - X)
            done = np.linalg.norm(Xn - X) <= 1e-13 * (1 + np.linalg.norm(X))
            X, t = Xn, tn
            if done:
                break
        r = Amat @ X.reshape(-1) - prob.b
        p = p + beta * r
        S = C + (Amat.T @ p).reshape(n, n)
        theta = max(-np.linalg.eigvalsh(S)[0], 0.0)
        pval = float(np.sum(C * X))
        dval = float(-prob.b @ p - prob.tau2 * theta)
        if np.linalg.norm(r) <= tol and abs(pval - dval) <= tol * (1 + abs(pval)):
            break
        beta = min(beta * 1.5, 1e6)
    return pval, dval, X, p
