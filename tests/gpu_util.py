"""Helpers shared by the GPU tests (test infrastructure)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def normwise(x, ref, terms):
    """||x - ref||_2 / ||terms||_2 where `terms` bounds the absolute
    contributions (sum of |summands| per entry)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = max(float(np.linalg.norm(terms)), 1e-300)
    return float(np.linalg.norm(x - ref)) / den


def abs_terms_T(prob, U):
    """Per-constraint sum of |(2 - delta) A_ij <U_i, U_j>| (plus |low-rank|)."""
    import oracle  # noqa
    w = np.where(prob.row == prob.col, 1.0, 2.0) * np.abs(prob.val)
    d = np.abs(np.einsum("kr,kr->k", U[prob.row], U[prob.col]))
    out = np.bincount(prob.con, weights=w * d, minlength=prob.m + 1)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        Y = K.T @ U
        out[l] += float(np.abs(D * (Y @ Y.T)).sum())
    return out


def abs_terms_W(prob, ptil, U):
    import scipy.sparse as sp
    v = np.abs(prob.val * np.asarray(ptil)[prob.con])
    off = prob.row != prob.col
    M = sp.csr_matrix((np.concatenate([v, v[off]]), (np.concatenate([prob.row, prob.col[off]]),
                                                     np.concatenate([prob.col, prob.row[off]]))),
                      shape=(prob.n, prob.n))
    out = M @ np.abs(U)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        out = out + abs(ptil[l]) * (np.abs(K) @ (np.abs(D) @ (np.abs(K).T @ np.abs(U))))
    return out
