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
    """Per-constraint sum of the absolute values of every product that forms
    T_l: sum over its entries of |(2 - delta) A_ij| sum_c |U_ic| |U_jc|, plus
    sum_ab |D_ab| (|K|^T |U|)_a . (|K|^T |U|)_b for a low-rank term."""
    A = np.abs(U)
    w = np.where(prob.row == prob.col, 1.0, 2.0) * np.abs(prob.val)
    d = np.einsum("kr,kr->k", A[prob.row], A[prob.col])
    out = np.bincount(prob.con, weights=w * d, minlength=prob.m + 1)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        Y = np.abs(K).T @ A
        out[l] += float((np.abs(D) * (Y @ Y.T)).sum())
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


def entrywise(x, ref, terms, tol, u):
    """max_k |x_k - ref_k| / (tol * terms_k + 4 u |ref_k|): <= 1 passes.
    `terms` is the per-entry sum of absolute contributions, u the unit
    roundoff of the stored result (an exact zero gets no slack)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = tol * np.asarray(terms, np.float64) + 4.0 * u * np.abs(ref)
    err = np.abs(x - ref)
    bad = err > 0
    if not bad.any():
        return 0.0
    return float(np.max(err[bad] / np.maximum(den[bad], 1e-300)))


U32, U64 = 2.0 ** -24, 2.0 ** -53


def cdp_terms(prob, U, ptil=None):
    """Error scales of the coded-diffraction operators (FFT rounding is
    normwise: a unitary transform of v errs by O(u log n) ||v||_2 in every
    entry).  For T: per constraint (l, k), 2 sum_c ||d_l u_c||_2 (|S_lkc| +
    ||d_l u_c||_2) with S the spectra; for W = A*(p~)U: per entry,
    sum_l |d_lj| max|y_l| ||d_l u_c||_2 plus the sparse part |C||U|."""
    L, nc = prob.cdp_masks.shape
    U = np.asarray(U, np.float64).reshape(prob.n, -1)
    Uc = U[:nc] + 1j * U[nc:]
    V = prob.cdp_masks[:, :, None] * Uc[None]
    nv = np.linalg.norm(V, axis=1)                           # (L, r)
    S = np.fft.fft(V, axis=1, norm="ortho")
    tT = np.zeros(prob.m + 1)
    tT[0] = float((U * U).sum())
    tT[1:] = (2.0 * nv[:, None, :] * (np.abs(S) + nv[:, None, :])).sum(axis=2).reshape(-1)
    if ptil is None:
        return tT
    y = np.abs(np.asarray(ptil)[1:]).reshape(L, nc).max(axis=1)      # (L,)
    half = (np.abs(prob.cdp_masks)[:, :, None] * (y[:, None] * nv)[:, None, :]).sum(axis=0)  # (nc, r)
    tW = np.vstack([half, half]) + abs(ptil[0]) * np.abs(U)
    return tT, tW
