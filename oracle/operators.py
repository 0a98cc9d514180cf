"""Oracle operators (FP64, numpy/scipy) — test infrastructure only.

Definitions followed (cuHALLaR paper, arXiv 2505.13719):
  * Section 1, eq. (Definition of Linear Operators): [A(X)]_l = A_l . X and
    A*(p) = sum_l p_l A_l.
  * Section 4, eq. (A tilde operator): A~(X) = (A_0 . X, A(X)) with A_0 = C and
    A~*(p~) = sum_{l=0}^m p~_l A_l for p~ = (1, p).
  * Section 3.2, eq. (HSLR-rep-body): A_l = A_l^sp + K_l D_l K_l^T.
  * Section 4.1, eq. (omega): because A_l^sp and UU^T are symmetric,
    A_l^sp . UU^T = sum_{i<=j} (2 - delta_ij) (A_l^sp)_ij <U_i, U_j>.
  * Section 2, eq. (AL function): L_beta(X; p) = C.X + p^T(A(X)-b) + beta/2 ||A(X)-b||^2.
  * Section 2, eq. (Grad U Space):
        grad_U L_beta(UU^T; p) = 2 [C + A*(p + beta (A(UU^T) - b))] U.
  * Section 5.4, eq. (phase retrieval SDP): constraints <a a^H, X> on a
    complex Hermitian X, here with coded-diffraction vectors: a_{l,k}^H u is
    the k-th entry of the unitary DFT of d_l * u.  The SDP is taken on its
    real form: a real column z of U is u = z[:n/2] + i z[n/2:], so that
    <a a^H, sum_c u_c u_c^H> = sum_c |a^H u_c|^2 (and Tr X = ||U||_F^2);
    the adjoint sum_k y_k a_k (a_k^H u) is D_l^H F^H (y_l * F D_l u).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _rowdot(U, i, j):
    return np.einsum("kr,kr->k", U[i], U[j])


def _cdp_spectra(prob, U):
    """F (d_l * u_c) for every pattern l and column c: shape (L, n_c, r)."""
    nc = prob.n // 2
    Uc = U[:nc] + 1j * U[nc:]
    return np.fft.fft(prob.cdp_masks[:, :, None] * Uc[None, :, :], axis=1, norm="ortho")


def a_tilde(prob, U):
    """T = A~(UU^T) in R^{m+1}: T_0 = C . UU^T and T_l = A_l . UU^T.

    Sparse part: sum over the listed upper-triangle entries of
    (2 - delta_ij) (A_l)_ij (UU^T)_ij (eq. omega); low-rank part:
    K D K^T . UU^T = Tr(D (K^T U)(K^T U)^T) (eq. T LR, cyclic trace).
    """
    U = np.asarray(U, np.float64).reshape(prob.n, -1)
    T = np.zeros(prob.m + 1)
    if prob.nnz:
        w = np.where(prob.row == prob.col, 1.0, 2.0) * prob.val
        T += np.bincount(prob.con, weights=w * _rowdot(U, prob.row, prob.col), minlength=prob.m + 1)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        Y = K.T @ U
        T[l] += float(np.sum(D * (Y @ Y.T)))
    if getattr(prob, "cdp_masks", None) is not None:
        # |a_{l,k}^H u_c|^2 summed over the columns, constraint l n_c + k
        T[1:] += (np.abs(_cdp_spectra(prob, U)) ** 2).sum(axis=2).reshape(-1)
    return T


def a_map(prob, U):
    """A(UU^T) in R^m (constraints l = 1..m only)."""
    return a_tilde(prob, U)[1:]


def adjoint_sparse(prob, ptilde):
    """Sparse symmetric matrix sum_l p~_l A_l^sp (pattern S union S^T)."""
    ptilde = np.asarray(ptilde, np.float64)
    v = prob.val * ptilde[prob.con]
    off = prob.row != prob.col
    rows = np.concatenate([prob.row, prob.col[off]])
    cols = np.concatenate([prob.col, prob.row[off]])
    vals = np.concatenate([v, v[off]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(prob.n, prob.n))


def adjoint_apply(prob, ptilde, U):
    """W = A~*(p~) U = (sum_l p~_l A_l) U, sparse plus low-rank parts
    (Section 4.2, eq. Adjoint calculation)."""
    U = np.asarray(U, np.float64)
    vec = U.ndim == 1
    U2 = U.reshape(prob.n, -1)
    W = adjoint_sparse(prob, ptilde) @ U2
    ptilde = np.asarray(ptilde, np.float64)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        W += ptilde[l] * (K @ (D @ (K.T @ U2)))
    if getattr(prob, "cdp_masks", None) is not None:
        L, nc = prob.cdp_masks.shape
        y = ptilde[1:].reshape(L, nc, 1)
        back = np.fft.ifft(y * _cdp_spectra(prob, U2), axis=1, norm="ortho")
        V = (np.conj(prob.cdp_masks)[:, :, None] * back).sum(axis=0)
        W += np.vstack([V.real, V.imag])
    return W.reshape(-1) if vec else W


def al_value(prob, U, p, beta):
    """g(U) = L_beta(UU^T; p); also returns T = A~(UU^T)."""
    T = a_tilde(prob, U)
    r = T[1:] - prob.b
    return float(T[0] + p @ r + 0.5 * beta * (r @ r)), T


def al_grad(prob, U, p, beta):
    """grad_U g(U) = 2 [C + A*(p + beta (A(UU^T) - b))] U."""
    T = a_tilde(prob, U)
    y = p + beta * (T[1:] - prob.b)
    return 2.0 * adjoint_apply(prob, np.concatenate([[1.0], y]), U)


def c_l1_norm(prob):
    """||C||_1 as the entrywise l1 norm of the full symmetric C (used in the
    dual-infeasibility term of eq. termination2).  The low-rank part is added
    densely for small n and by its exact value for the all-ones K."""
    sel = prob.con == 0
    if sel.any():
        Csp = sp.coo_matrix((prob.val[sel], (prob.row[sel], prob.col[sel])), shape=(prob.n, prob.n)).tocsr()
        Csp = Csp + sp.triu(Csp, k=1).T
    else:
        Csp = sp.csr_matrix((prob.n, prob.n))
    lr = [(K, D) for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D) if l == 0]
    if not lr:
        return float(np.abs(Csp).sum())
    if prob.n <= 4096:
        dense = Csp.toarray()
        for K, D in lr:
            dense = dense + K @ D @ K.T
        return float(np.abs(dense).sum())
    # large n: only the rank-1 all-ones form c e e^T plus a sparse part is supported
    (K, D), = lr
    assert K.shape[1] == 1 and np.all(K == 1.0) and Csp.nnz == 0
    return float(abs(D[0, 0]) * prob.n * prob.n)
