"""Oracle HALLaR solver (FP64, numpy) — test infrastructure only.

Follows the cuHALLaR paper (arXiv 2505.13719) step by step:
  * Alg. 1 (HALLaR): outer augmented-Lagrangian loop over t, the HLR while
    loop (nonconvex solve, minimum eigenpair of G, Frank-Wolfe gap test,
    Frank-Wolfe step), the multiplier update (eq. dual update SDP Algo 2).
  * Appendix A (ADAP-AIPP) and Appendix A.1 (ADAP-FISTA) for the nonconvex
    solve.
  * Section 5.1 (eq. termination2) for the relative stopping test and
    "Initialization" for U_0 (passed in by the caller, projected onto B_tau).

Readings where the paper is silent (the GPU solver uses the same numbers,
defined on its own side):
  * beta_1 = 1; after outer iteration t (the paper only says "adaptive,
    LANCELOT-like", Section 2): beta <- min(4 beta, beta_max) when
    ||A(X_t) - b|| > 0.5 ||A(X_{t-1}) - b|| and the relative infeasibility is
    at least 0.1 times the larger of the relative gap and dual infeasibility,
    16 beta when ||A(X_t) - b|| > 0.9 ||A(X_{t-1}) - b||; otherwise beta is
    kept.  beta_max = 1e16 only guards against overflow: the penalty an
    instance needs scales with its data (the Lovasz theta SDP of an n-vertex
    graph of degree d needs multipliers of order n/d on residuals of order
    1/n, so beta near n^2: about 1.7e7 for the 12-cube, 1e12 for the 20-cube).
  * eps_t = max(eps1 * 0.5^(t-1), eps_floor) * (1 + max(|pval_{t-1}|, |g_t(U_{t-1})|))
    with eps1 = 1e-2, eps_floor = 0.2 * eps (pval_0 = C . U_0 U_0^T; the AL
    value at the start of the outer iteration keeps the scale right when the
    random start has a tiny objective); the stationarity tolerance handed
    to ADAP-AIPP is rho_t = eps_t (the tolerance Alg. 1 passes to its
    nonconvex solver) divided by tau: G . YY^T = <grad g(Y), Y>/2 moves by up
    to tau ||R|| / 2 when the stationarity residual is R, so rho_t = eps_t / tau
    makes the two tolerances commensurate (the paper's Alg. 1 hands eps_t to
    both; tau = 1 for theta, where the readings coincide).
  * sigma = 0.3, chi = 1e-3, lambda_0 = 10 for the first call, later calls
    start from the last accepted prox stepsize; M_j = max(1, Mbar_{j-1}/2).
    The descent check (eq. subdiff ineq check) allows a slack of
    1e-13 (1 + |lambda g(W_{j-1})|) for rounding.
  * V of ADAP-FISTA's output: V = grad psi_s(y) - grad psi_s(x~) + L (x~ - y),
    and the linearisation l_psi(u; x~) = psi_s(x~) + <grad psi_s(x~), u - x~>.
  * theta = 0 gives y = 0: the Frank-Wolfe step then shrinks Y without adding
    a column; a zero denominator in the step size gives alpha = 1.
  * After every nonconvex solve, Y is rotated onto the eigenvectors of
    Y^T Y and directions with sigma^2 <= 1e-14 sigma_max^2 are dropped (Y Y^T
    unchanged up to that size).  Rank cap: when the Frank-Wolfe iterate has
    more columns than the cap, its numerically null directions are dropped;
    if it still has too many, the solve stops with status "rank_cap" and
    returns the iterate before the step (the cap is never met silently).
    With rank_cap_truncate only the cap largest directions are kept instead,
    and each such truncation is counted.
  * Eigen solve: Lanczos stops once the Ritz residual is
    <= eig_frac * eps_t / tau^2 (floor 1e-13 max(1, |lambda|)), so that the
    error it puts into the gap G.YY^T + tau^2 theta stays below eig_frac eps_t.
  * dinf = max(0, -(lambda_hat - res + theta))/(1 + ||C||_1) where
    (lambda_hat, res) is the Ritz value and residual of the last eigen solve
    on G = C + A*(p_t).
  * Certification of lambda_min: once the three relative errors pass, one
    more Lanczos run on G = C + A*(p_t), started from a fresh Gaussian vector
    and limited to cert_max_iter products, is made; if its Ritz value is
    smaller, theta, dval, gap and dinf are recomputed with it and the test is
    repeated.  Both Ritz values bound lambda_min from above, so this can only
    tighten the dual value (near the optimum the smallest eigenvalues of G
    cluster, one per primal column, and the warm-started run can settle on a
    member above the minimum).
  * Objective accuracy: besides the three relative errors, the solve stops
    only when |pval - dval| + |p_t^T (A(X_t) - b)| <= eps (1 + |pval|).  The
    relative gap of eq. termination2 divides by 1 + |pval| + |dval|, about
    twice the objective, so on its own it allows an objective error near
    2 eps.  Weak duality puts P* above dval, pval lies above dval - |p^T r|,
    and P* <= pval + p*^T r for an optimal multiplier p*, so with p_t close to
    p* the bound limits |pval - P*| to eps relative (obj_check = False drops
    it).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from .operators import a_tilde, adjoint_apply, c_l1_norm
from .lanczos import min_eig


@dataclass
class Options:
    eps: float = 1e-5
    beta1: float = 1.0
    beta_growth: float = 4.0
    beta_max: float = 1e16
    beta_rule: str = "ratio"
    infeas_ratio: float = 0.5
    pinf_gate: float = 0.1
    stall_ratio: float = 0.9        # ||r_t|| above this fraction of ||r_{t-1}||: growth stall_growth
    stall_growth: float = 16.0
    balance: float = 3.0
    rho_over_tau: bool = True
    beta_min: float = 1e-3
    eps1: float = 1e-2
    eps_floor: float = 0.2          # times eps
    eps_decay: float = 0.5
    sigma: float = 0.3
    chi: float = 1e-3
    lam0: float = 10.0
    lam_grow: float = 1.0
    fista_max_iter: int = 2000
    aipp_max_iter: int = 500
    hlr_max_iter: int = 1000
    outer_max_iter: int = 300
    eig_tol: float = 1e-13
    eig_frac: float = 0.1
    eig_kmax: int = 80
    cert_max_iter: int = 400        # matvecs of the cold-started certification run (0: none)
    obj_check: bool = True          # also stop only when |pval - dval| + |p^T r| <= eps (1 + |pval|)
    rank_cap: int = 0               # 0: unbounded
    rank_cap_truncate: bool = False  # at the cap: keep the largest directions (else stop, status "rank_cap")
    drop_tol: float = 1e-14
    time_limit: float = 3600.0
    seed: int = 0                   # eigen start vectors


@dataclass
class Result:
    status: str
    U: np.ndarray
    p: np.ndarray
    theta: float
    pval: float
    dval: float
    pinf: float
    gap: float
    dinf: float
    rank: int
    outer_iters: int
    counters: dict = field(default_factory=dict)
    history: list = field(default_factory=list)


def _proj_ball(U, tau):
    """Euclidean projection onto B_tau = {U : ||U||_F <= tau} (eq. dimensional ball)."""
    nrm = np.linalg.norm(U)
    return U if nrm <= tau else U * (tau / nrm)


class ALFunction:
    """g(U) = L_beta(UU^T; p) with counters of operator evaluations."""

    def __init__(self, prob, p, beta, counters):
        self.prob, self.p, self.beta, self.c = prob, p, beta, counters

    def eval(self, U):
        """(g(U), T = A~(UU^T), y' = p + beta (A(UU^T) - b))."""
        self.c["sddmm"] += 1
        T = a_tilde(self.prob, U)
        r = T[1:] - self.prob.b
        g = float(T[0] + self.p @ r + 0.5 * self.beta * (r @ r))
        return g, T, self.p + self.beta * r

    def grad_from(self, U, y):
        """grad g(U) = 2 (C + A*(y)) U for y = y'(U) (eq. Grad U Space)."""
        self.c["spmm"] += 1
        return 2.0 * adjoint_apply(self.prob, np.concatenate([[1.0], y]), U)


class _Psi:
    """psi_s(u) = lam g(u) + 1/2 ||u - W||^2 (eq. psi s)."""

    def __init__(self, g, lam, W):
        self.g, self.lam, self.W = g, lam, W

    def value(self, u):
        gv, _, _ = self.g.eval(u)
        d = u - self.W
        return self.lam * gv + 0.5 * float(np.vdot(d, d)), gv

    def value_grad(self, u):
        gv, _, y = self.g.eval(u)
        d = u - self.W
        return self.lam * gv + 0.5 * float(np.vdot(d, d)), self.lam * self.g.grad_from(u, y) + d


def fista(psi, x0, mu, L0, sigma, chi, tau, max_iter, counters):
    """ADAP-FISTA (Appendix A.1).  Returns (ok, y, V, L, g(y))."""
    y = x0.copy()
    x = x0.copy()
    A, tk, L = 0.0, 1.0, float(L0)
    for i in range(max_iter):
        # gradient step from the extrapolated point, doubling L until the
        # descent inequality holds
        for _ in range(200):
            counters["fista_trials"] += 1
            a = (tk + math.sqrt(tk * tk + 4.0 * tk * A * (L - mu))) / (2.0 * (L - mu))
            xt = (A * y + a * x) / (A + a)
            f_xt, g_xt = psi.value_grad(xt)
            y_new = _proj_ball(xt - g_xt / L, tau)
            f_y, gy = psi.value(y_new)
            d = y_new - xt
            dd = float(np.vdot(d, d))
            lin = f_xt + float(np.vdot(g_xt, d))
            if lin + 0.25 * (1.0 - chi) * L * dd >= f_y:
                break
            L *= 2.0
        else:
            return False, None, None, L, None
        # updates of A, tau, s and x
        A_new = A + a
        tk_new = tk + a * mu
        s = (L - mu) * (xt - y_new)
        x = (mu * a * y_new + tk * x - a * s) / tk_new
        e = y_new - x0
        ee = float(np.vdot(e, e))
        # failure test
        if ee < chi * A_new * L * dd:
            return False, None, None, L, None
        # success test
        if math.sqrt(float(np.vdot(s, s))) <= sigma * math.sqrt(ee):
            _, g_y = psi.value_grad(y_new)
            V = g_y - g_xt + L * (xt - y_new)
            return True, y_new, V, L, gy
        y, A, tk = y_new, A_new, tk_new
    return False, None, None, L, None


def aipp(g, W0, g0, lam0, rho, opts, tau, counters):
    """ADAP-AIPP (Appendix A).  Returns (status, W, R, lam, g(W))."""
    W_prev, g_prev = W0, g0
    lam, Mbar = float(lam0), 1.0
    for j in range(opts.aipp_max_iter):
        counters["aipp_iters"] += 1
        while True:
            Mj = max(1.0, 0.5 * Mbar)
            psi = _Psi(g, lam, W_prev)
            ok, W, V, L, gW = fista(psi, W_prev, 0.5, Mj, opts.sigma, opts.chi, tau,
                                    opts.fista_max_iter, counters)
            if ok:
                dW = W - W_prev
                lhs = lam * g_prev - (lam * gW + 0.5 * float(np.vdot(dW, dW)))
                # eq. (subdiff ineq check), with a rounding-level slack
                if lhs >= float(np.vdot(V, -dW)) - 1e-13 * (1.0 + abs(lam * g_prev)):
                    break
            lam *= 0.5
            counters["lam_halvings"] += 1
            if lam < 1e-30:
                return "numerical", W_prev, None, lam, g_prev
        R = (V + W_prev - W) / lam
        Mbar = L
        W_prev, g_prev = W, gW
        if np.linalg.norm(R) <= rho:
            return "ok", W, R, lam, gW
    return "iter_limit", W_prev, None, lam, g_prev


def fw_alpha(gap, AYY, Ayy, tau2, beta):
    """Exact line search of the Frank-Wolfe step (eq. FW stepsize):
    alpha = min{gap / (beta ||A(YY^T) - A(tau^2 y y^T)||^2), 1}, where gap =
    G.YY^T + tau^2 theta is minus the slope and beta ||.||^2 the curvature of
    alpha -> L_beta((1-alpha) YY^T + alpha tau^2 y y^T; p)."""
    diff = AYY - tau2 * Ayy
    den = beta * float(diff @ diff)
    return 1.0 if den <= 0.0 else min(gap / den, 1.0)


def fw_step(Y, y, theta, alpha, tau):
    """Frank-Wolfe update in U-space (eq. tilde Y Algo 2): (tau y, 1) if
    alpha = 1, else [sqrt(1-alpha) Y, sqrt(alpha) tau y]; with y = 0
    (theta = 0) no column is added."""
    if alpha >= 1.0:
        return (tau * y).reshape(-1, 1)
    if theta <= 0.0:
        return math.sqrt(1.0 - alpha) * Y
    return np.hstack([math.sqrt(1.0 - alpha) * Y, (math.sqrt(alpha) * tau * y).reshape(-1, 1)])


def metrics(prob, pval, dval, T_Y, lam_min_S, cnorm1):
    """Relative errors of eq. termination2 (Section 5.1)."""
    r = T_Y[1:] - prob.b
    pinf = float(np.linalg.norm(r)) / (1.0 + float(np.abs(prob.b).sum()))
    gap = abs(pval - dval) / (1.0 + abs(pval) + abs(dval))
    dinf = max(0.0, -lam_min_S) / (1.0 + cnorm1)
    return pinf, gap, dinf


def _compress(Y, drop_tol, keep_max=0):
    """Rotate Y onto the eigenvectors of Y^T Y (Y Q Q^T Y^T = Y Y^T) and drop
    the directions whose squared singular value is <= drop_tol * sigma_max^2;
    with keep_max > 0 at most the keep_max largest directions are kept."""
    G = Y.T @ Y
    w, Q = np.linalg.eigh(G)
    keep = w > drop_tol * max(w[-1], 0.0)
    if keep_max and keep.sum() > keep_max:
        keep[: w.size - keep_max] = False
    if keep.all():
        return Y
    if not keep.any():
        keep[-1] = True
    return Y @ Q[:, keep]


def hallar(prob, U0, opts: Options = None, p0=None):
    """HALLaR (Alg. 1) with ADAP-AIPP as the nonconvex solver."""
    opts = opts or Options()
    t_start = time.time()
    n = prob.n
    tau = math.sqrt(prob.tau2)
    rng = np.random.default_rng(opts.seed)
    counters = dict(sddmm=0, spmm=0, matvec=0, fista_trials=0, aipp_iters=0,
                    lam_halvings=0, hlr_iters=0, eig_calls=0, truncations=0, aipp_caps=0)
    cn1 = c_l1_norm(prob)
    U = _proj_ball(np.asarray(U0, np.float64).reshape(n, -1), tau)   # U_0 in B_tau
    p = np.zeros(prob.m) if p0 is None else np.asarray(p0, np.float64).copy()
    beta = opts.beta1
    lam = opts.lam0
    T0 = a_tilde(prob, U)
    pval_prev = float(T0[0])
    rnorm_prev = float(np.linalg.norm(T0[1:] - prob.b))
    v_prev = None
    history = []
    status = "iter_limit"
    theta = 0.0
    pval = dval = pinf = gap = dinf = float("nan")
    for t in range(1, opts.outer_max_iter + 1):
        g = ALFunction(prob, p, beta, counters)
        Yt = U
        gY, _, _ = g.eval(Yt)
        scale = 1.0 + max(abs(pval_prev), abs(gY))
        eps_t = max(opts.eps1 * opts.eps_decay ** (t - 1), opts.eps_floor * opts.eps) * scale
        rho = eps_t / (max(1.0, tau) if opts.rho_over_tau else 1.0)
        hlr_ok = False
        for _ in range(opts.hlr_max_iter):
            counters["hlr_iters"] += 1
            st, Y, R, lam, gY = aipp(g, Yt, gY, min(lam * opts.lam_grow, opts.lam0), rho, opts, tau, counters)
            if st == "numerical":
                status = st
                break
            # st == "iter_limit": the safeguard on ADAP-AIPP's iterations (the
            # paper's method has none) hands back its last iterate, which the
            # Frank-Wolfe certificate below then judges like any other
            if st != "ok":
                counters["aipp_caps"] += 1
            if Y.shape[1] > 1:
                Y = _compress(Y, opts.drop_tol)
            # G = C + A*(p + beta (A(YY^T) - b)) (eq. Grad X Space)
            _, TY, yG = g.eval(Y)
            ptil = np.concatenate([[1.0], yG])

            def matvec(v, _pt=ptil):
                counters["matvec"] += 1
                return adjoint_apply(prob, _pt, v)

            start = rng.standard_normal(n)
            if v_prev is not None:
                start = v_prev + 1e-2 * start / math.sqrt(n)
            counters["eig_calls"] += 1
            lmin, v, einfo = min_eig(matvec, n, start, tol=opts.eig_tol, kmax=opts.eig_kmax,
                                    atol=opts.eig_frac * eps_t / prob.tau2)
            v_prev = v
            theta = max(-lmin, 0.0)
            y = v if theta > 0.0 else np.zeros(n)
            GY = adjoint_apply(prob, ptil, Y)
            counters["spmm"] += 1
            gap_fw = float(np.vdot(GY, Y)) + prob.tau2 * theta
            if gap_fw <= eps_t:
                hlr_ok = True
                break
            alpha = fw_alpha(gap_fw, TY[1:], a_tilde(prob, y.reshape(n, 1))[1:], prob.tau2, beta)
            Yt = fw_step(Y, y, theta, alpha, tau)
            if opts.rank_cap and Yt.shape[1] > opts.rank_cap:
                # rank cap: drop numerically null directions; if the step still
                # needs more columns, stop ("rank_cap", the iterate before the
                # step is returned) unless truncation was asked for
                if opts.rank_cap_truncate:
                    counters["truncations"] += 1
                    Yt = _compress(Yt, opts.drop_tol, opts.rank_cap)
                else:
                    Yt = _compress(Yt, opts.drop_tol)
                    if Yt.shape[1] > opts.rank_cap:
                        status = "rank_cap"
                        break
            gY, _, _ = g.eval(Yt)
        else:
            status = "iter_limit"
        if not hlr_ok:
            U = Y if st == "ok" or status == "rank_cap" else U
            break
        # U_t = Y; p_t = p + beta (A(U_t U_t^T) - b)  (eq. dual update SDP Algo 2)
        U = Y
        p = yG
        pval = float(TY[0])
        dval = float(-prob.b @ p - prob.tau2 * theta)
        lam_S = (lmin - einfo["residual"]) + theta
        pinf, gap, dinf = metrics(prob, pval, dval, TY, lam_S, cn1)
        rnorm = float(np.linalg.norm(TY[1:] - prob.b))
        if max(pinf, gap, dinf) <= opts.eps and opts.cert_max_iter > 0:
            # certification: the Ritz value bounds lambda_min(C + A*(p_t)) from
            # above, and a warm-started run can stop on a member of the cluster
            # of smallest eigenvalues above the minimum; one cold-started run
            # takes the smaller Ritz value (theta and dval only tighten)
            counters["eig_calls"] += 1
            lc, _, ci = min_eig(matvec, n, rng.standard_normal(n), tol=opts.eig_tol, kmax=opts.eig_kmax,
                                max_restarts=max(1, opts.cert_max_iter // max(2, min(opts.eig_kmax, n))),
                                atol=opts.eig_frac * eps_t / prob.tau2)
            if lc < lmin:
                lmin, theta = lc, max(-lc, 0.0)
                dval = float(-prob.b @ p - prob.tau2 * theta)
                pinf, gap, dinf = metrics(prob, pval, dval, TY, (lc - ci["residual"]) + theta, cn1)
        # a-posteriori estimate of |pval - P*| (objective accuracy test)
        objb = abs(pval - dval) + abs(float(p @ (TY[1:] - prob.b)))
        history.append(dict(t=t, beta=beta, rank=U.shape[1], pval=pval, dval=dval, pinf=pinf,
                            gap=gap, dinf=dinf, eps_t=eps_t, theta=theta, objb=objb))
        if max(pinf, gap, dinf) <= opts.eps and (not opts.obj_check or objb <= opts.eps * (1.0 + abs(pval))):
            status = "ok"
            break
        if time.time() - t_start > opts.time_limit:
            status = "time_limit"
            break
        if opts.beta_rule == "ratio":
            # LANCELOT-like: raise the penalty when the infeasibility did not
            # drop by the factor infeas_ratio since the previous outer iteration
            if rnorm > opts.infeas_ratio * rnorm_prev and pinf > opts.pinf_gate * max(gap, dinf):
                grow = opts.stall_growth if rnorm > opts.stall_ratio * rnorm_prev else opts.beta_growth
                beta = min(beta * grow, opts.beta_max)
        else:
            if pinf > opts.balance * max(gap, dinf):
                beta = min(beta * opts.beta_growth, opts.beta_max)
            elif max(gap, dinf) > opts.balance * pinf:
                beta = max(beta / opts.beta_growth, opts.beta_min)
        rnorm_prev = rnorm
        pval_prev = pval
    return Result(status=status, U=U, p=p, theta=theta, pval=pval, dval=dval, pinf=pinf,
                  gap=gap, dinf=dinf, rank=int(U.shape[1]), outer_iters=len(history),
                  counters=counters, history=history)
