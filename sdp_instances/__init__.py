"""Seeded synthetic SDP instances (data only).

This module turns graphs and planted matrices into the input data of the
primal problem (P) of the cuHALLaR paper (Section 1):

    min C . X   s.t.  A_l . X = b_l (l = 1..m),  Tr X <= tau^2,  X PSD.

Every data matrix A_l (with A_0 = C) is given in the hybrid sparse/low-rank
form of Section 3.2 (eq. HSLR-rep-body): a sparse symmetric part listed by
its upper-triangle entries (i <= j) plus an optional low-rank part K D K^T.

It holds none of the solver's arithmetic: it only writes down instances.
Both the CPU oracle and the GPU library consume the `Problem` objects built
here; neither is imported by this module.

Workload recipes (the paper's own graph files are not available, so these
seeded generators stand in for them with the same shapes):
  * MaxCut SDP (diag X = 1, C = -Laplacian/4) on Erdos-Renyi graphs and on
    2-D tori, unit or +-1 edge weights;
  * Lovasz theta SDP (Section 5.3, eq. lovasz) on Erdos-Renyi graphs and on
    small graphs with known theta;
  * matrix-completion SDP (Section 5.2, eq. matcomp-sdp) with a planted
    Gaussian rank-r target.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Problem", "er_edges", "torus_edges", "cycle_edges", "complete_edges",
    "petersen_edges", "hypercube_edges", "pm1_weights", "maxcut_problem",
    "theta_problem", "mc_problem", "mc_count_tables", "gaussian_u0",
    "random_hslr", "maxcut_er_800", "maxcut_torus", "theta_er",
    "mc_planted", "served_stream_sizes", "served_request",
]


@dataclass
class Problem:
    """One SDP instance in HSLR form.

    Sparse part: entries (row[k], col[k], con[k], val[k]) with
    row[k] <= col[k] (upper triangle), con[k] in [0, m] (0 is the objective
    C = A_0) and val[k] = (A_con)_{row,col}.  Duplicated (i, j, l) triples
    are summed.  Low-rank part: for each t, A_{lr_con[t]} += K_t D_t K_t^T
    with K_t of shape (n, r_t) and D_t symmetric (r_t, r_t).
    """

    name: str
    n: int
    m: int
    tau2: float
    row: np.ndarray
    col: np.ndarray
    con: np.ndarray
    val: np.ndarray
    b: np.ndarray
    lr_con: List[int] = field(default_factory=list)
    lr_K: List[np.ndarray] = field(default_factory=list)
    lr_D: List[np.ndarray] = field(default_factory=list)
    meta: dict = field(default_factory=dict)
    # coded-diffraction constraints of complex phase retrieval (Section 5.4),
    # stated on the real form of the complex Hermitian variable: n = 2 n_c,
    # a real column z of U is the complex vector u = z[:n_c] + i z[n_c:], and
    # constraint l n_c + k (0-based) is sum_c |(F (d_l * u_c))_k|^2 with F
    # the unitary n_c-point DFT and d_l = cdp_masks[l]; there are m = L n_c
    # of them and no sparse or low-rank constraint entries
    cdp_masks: Optional[np.ndarray] = None

    def __post_init__(self):
        self.row = np.ascontiguousarray(self.row, dtype=np.int64)
        self.col = np.ascontiguousarray(self.col, dtype=np.int64)
        self.con = np.ascontiguousarray(self.con, dtype=np.int64)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        self.lr_K = [np.ascontiguousarray(K, dtype=np.float64).reshape(self.n, -1) for K in self.lr_K]
        self.lr_D = [np.ascontiguousarray(D, dtype=np.float64) for D in self.lr_D]
        assert self.row.shape == self.col.shape == self.con.shape == self.val.shape
        assert self.b.shape == (self.m,)
        if self.row.size:
            assert (self.row <= self.col).all(), "entries must be upper-triangular (i <= j)"
            assert self.row.min() >= 0 and self.col.max() < self.n
            assert self.con.min() >= 0 and self.con.max() <= self.m
        if self.cdp_masks is not None:
            self.cdp_masks = np.ascontiguousarray(self.cdp_masks, dtype=np.complex128)
            L, nc = self.cdp_masks.shape
            assert self.n == 2 * nc and self.m == L * nc
            assert not self.lr_con and (self.con == 0).all(), "coded-diffraction problems take C only as entries"

    @property
    def nnz(self) -> int:
        return int(self.row.size)


# ---------------------------------------------------------------- graphs

def er_edges(n: int, p: float, rng: np.random.Generator):
    """Edges (i < j) of an Erdos-Renyi G(n, p) graph.

    Every unordered pair is kept independently with probability p; the kept
    pairs are found by geometric skips over the row-major list of the
    n(n-1)/2 pairs, which is exact for Bernoulli(p) selection.
    """
    N = n * (n - 1) // 2
    if N == 0 or p <= 0.0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if p >= 1.0:
        return complete_edges(n)
    chunks = []
    pos = -1
    batch = int(N * p + 8 * math.sqrt(N * p) + 64)
    while True:
        idx = pos + np.cumsum(rng.geometric(p, size=batch).astype(np.int64))
        keep = idx[idx < N]
        chunks.append(keep)
        if keep.size < idx.size:
            break
        pos = int(idx[-1])
    k = np.concatenate(chunks)
    # linear index k -> (i, j): row i starts at i*(2n-i-1)/2
    twon1 = 2 * n - 1
    i = np.floor((twon1 - np.sqrt(float(twon1) ** 2 - 8.0 * k)) / 2.0).astype(np.int64)
    start = i * (twon1 - i) // 2
    # repair floating-point rounding of the square root
    lo = k < start
    while lo.any():
        i[lo] -= 1
        start = i * (twon1 - i) // 2
        lo = k < start
    nxt = (i + 1) * (twon1 - i - 1) // 2
    hi = k >= nxt
    while hi.any():
        i[hi] += 1
        start = i * (twon1 - i) // 2
        nxt = (i + 1) * (twon1 - i - 1) // 2
        hi = k >= nxt
    j = k - start + i + 1
    return i, j


def torus_edges(k1: int, k2: int):
    """2-D periodic grid: vertex v = k2*row + col, edges to the right and down
    neighbours (each vertex has degree 4 when k1, k2 >= 3)."""
    v = np.arange(k1 * k2, dtype=np.int64)
    r, c = v // k2, v % k2
    right = r * k2 + (c + 1) % k2
    down = ((r + 1) % k1) * k2 + c
    a = np.concatenate([v, v])
    b = np.concatenate([right, down])
    i, j = np.minimum(a, b), np.maximum(a, b)
    keep = i != j
    i, j = i[keep], j[keep]
    # k = 2 along an axis would list the same edge twice
    key = np.unique(i * (k1 * k2) + j)
    return key // (k1 * k2), key % (k1 * k2)


def cycle_edges(n: int):
    i = np.arange(n, dtype=np.int64)
    j = (i + 1) % n
    return np.minimum(i, j), np.maximum(i, j)


def complete_edges(n: int):
    i, j = np.triu_indices(n, k=1)
    return i.astype(np.int64), j.astype(np.int64)


def petersen_edges():
    outer = [(k, (k + 1) % 5) for k in range(5)]
    spokes = [(k, k + 5) for k in range(5)]
    inner = [(5 + k, 5 + (k + 2) % 5) for k in range(5)]
    e = np.array(outer + spokes + inner, dtype=np.int64)
    return np.minimum(e[:, 0], e[:, 1]), np.maximum(e[:, 0], e[:, 1])


def hypercube_edges(d: int):
    """Hamming graph H(d, 2): vertices are d-bit words, edges join words at
    Hamming distance 1; |E| = 2^d d / 2."""
    n = 1 << d
    v = np.arange(n, dtype=np.int64)
    ii, jj = [], []
    for bit in range(d):
        u = v ^ (1 << bit)
        keep = v < u
        ii.append(v[keep])
        jj.append(u[keep])
    return np.concatenate(ii), np.concatenate(jj)


def pm1_weights(count: int, rng: np.random.Generator):
    return np.where(rng.random(count) < 0.5, -1.0, 1.0)


# ---------------------------------------------------------------- problems

def maxcut_problem(n: int, i, j, w=None, name: str = "maxcut") -> Problem:
    """MaxCut SDP: min C . X, X_ll = 1 (l = 1..n), X PSD, with C = -L/4 and
    L = Diag(W 1) - W the weighted Laplacian; tau^2 = n (Tr X = n is implied
    by the diagonal constraints).  The SDP value -pval upper-bounds the
    maximum cut."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    w = np.ones(i.size) if w is None else np.asarray(w, np.float64)
    deg = np.bincount(i, weights=w, minlength=n) + np.bincount(j, weights=w, minlength=n)
    diag = np.arange(n, dtype=np.int64)
    nzd = deg != 0.0
    row = np.concatenate([i, diag[nzd], diag])
    col = np.concatenate([j, diag[nzd], diag])
    con = np.concatenate([np.zeros(i.size, np.int64), np.zeros(int(nzd.sum()), np.int64), diag + 1])
    val = np.concatenate([w / 4.0, -deg[nzd] / 4.0, np.ones(n)])
    return Problem(name=name, n=n, m=n, tau2=float(n), row=row, col=col, con=con,
                   val=val, b=np.ones(n),
                   meta={"kind": "maxcut", "edges": int(i.size)})


def theta_problem(n: int, i, j, name: str = "theta") -> Problem:
    """Lovasz theta SDP (eq. lovasz) as a minimisation: C = -e e^T (low rank,
    K = e, D = [-1]), one constraint X_ij = 0 per edge written as
    A_l = (E_ij + E_ji)/2, and Tr X <= 1 (tau^2 = 1).  pval = -theta(G)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    m = int(i.size)
    return Problem(name=name, n=n, m=m, tau2=1.0, row=i, col=j,
                   con=np.arange(1, m + 1, dtype=np.int64), val=np.full(m, 0.5),
                   b=np.zeros(m), lr_con=[0], lr_K=[np.ones((n, 1))],
                   lr_D=[np.array([[-1.0]])],
                   meta={"kind": "theta", "edges": m})


def mc_problem(n1: int, n2: int, ii, jj, Mvals, tau2: float, name: str = "mc") -> Problem:
    """Matrix-completion SDP (eq. matcomp-sdp): X = [[W1, Y], [Y^T, W2]],
    min Tr(X)/2 s.t. Y_ij = M_ij on the observed set.  C = I/2 is sparse
    (diagonal), each observation is A_l = (E_{i,n1+j} + E_{n1+j,i})/2 with
    b_l = M_ij."""
    n = n1 + n2
    ii = np.asarray(ii, np.int64)
    jj = np.asarray(jj, np.int64)
    m = int(ii.size)
    d = np.arange(n, dtype=np.int64)
    row = np.concatenate([d, ii])
    col = np.concatenate([d, n1 + jj])
    con = np.concatenate([np.zeros(n, np.int64), np.arange(1, m + 1, dtype=np.int64)])
    val = np.concatenate([np.full(n, 0.5), np.full(m, 0.5)])
    return Problem(name=name, n=n, m=m, tau2=float(tau2), row=row, col=col, con=con,
                   val=val, b=np.asarray(Mvals, np.float64),
                   meta={"kind": "mc", "n1": n1, "n2": n2})


def mc_count_tables(n1: int, n2: int, r: int) -> int:
    """Number of observed entries used by every row of the paper's
    matrix-completion table (Table tab:gpuourmethod_vs_cpu):
    ceil(gamma * r * (n1 + n2)) with oversampling gamma = r * ln(n1 + n2)."""
    return int(math.ceil(r * math.log(n1 + n2) * r * (n1 + n2)))


def gaussian_u0(n: int, seed: int, cols: int = 1) -> np.ndarray:
    """Initial factor of Section 5.1 ("Initialization"): an n x cols matrix of
    independent standard Gaussians (cols = 1 in the paper)."""
    return np.random.default_rng(seed).standard_normal((n, cols))


def random_hslr(n: int, m: int, seed: int, nnz: int = 0, lowrank: bool = True,
                lowrank_nonobjective: bool = False) -> Problem:
    """Small random HSLR instance for operator tests: random symmetric sparse
    entries spread over C and m constraints, duplicated triples, pairs shared
    by several constraints, constraints with several entries, diagonal
    entries and (optionally) a low-rank objective term."""
    rng = np.random.default_rng(seed)
    nnz = nnz or 4 * (n + m)
    a = rng.integers(0, n, nnz)
    b_ = rng.integers(0, n, nnz)
    row, col = np.minimum(a, b_), np.maximum(a, b_)
    con = rng.integers(0, m + 1, nnz)
    # make sure every constraint has at least one entry
    extra = np.arange(1, m + 1)
    ea = rng.integers(0, n, m)
    eb = rng.integers(0, n, m)
    row = np.concatenate([row, np.minimum(ea, eb), row[:5]])
    col = np.concatenate([col, np.maximum(ea, eb), col[:5]])
    con = np.concatenate([con, extra, con[:5]])           # last 5 duplicate triples
    val = rng.standard_normal(row.size)
    lr_con, lr_K, lr_D = [], [], []
    if lowrank:
        r0 = 2
        K = rng.standard_normal((n, r0))
        D = rng.standard_normal((r0, r0))
        lr_con.append(0); lr_K.append(K); lr_D.append(D + D.T)
    if lowrank_nonobjective:
        K = rng.standard_normal((n, 1))
        lr_con.append(int(rng.integers(1, m + 1))); lr_K.append(K); lr_D.append(np.array([[0.7]]))
    bvec = rng.standard_normal(m)
    return Problem(name=f"rand{n}x{m}s{seed}", n=n, m=m, tau2=float(n), row=row, col=col,
                   con=con, val=val, b=bvec, lr_con=lr_con, lr_K=lr_K, lr_D=lr_D,
                   meta={"kind": "random"})


# ---------------------------------------------------------------- workloads

def maxcut_er_800(seed: int = 1) -> Problem:
    """MaxCut SDP on G(n = 800, p = 0.02) with unit weights."""
    rng = np.random.default_rng(seed)
    i, j = er_edges(800, 0.02, rng)
    return maxcut_problem(800, i, j, name=f"maxcut_er800_s{seed}")


def maxcut_torus(k1: int = 1000, k2: int = 1000, seed: int = 2, unit: bool = False) -> Problem:
    """MaxCut SDP on a k1 x k2 torus (4-regular), weights +-1 uniform (or 1)."""
    i, j = torus_edges(k1, k2)
    w = np.ones(i.size) if unit else pm1_weights(i.size, np.random.default_rng(seed))
    return maxcut_problem(k1 * k2, i, j, w, name=f"maxcut_torus{k1}x{k2}_{'unit' if unit else 's%d' % seed}")


def theta_er(n: int = 50_000, avg_deg: float = 10.0, seed: int = 3) -> Problem:
    """Lovasz theta SDP on G(n, avg_deg/(n-1))."""
    rng = np.random.default_rng(seed)
    i, j = er_edges(n, avg_deg / (n - 1), rng)
    return theta_problem(n, i, j, name=f"theta_er{n}_s{seed}")


def mc_planted(n1: int, n2: int, r: int, m: int, seed: int = 4) -> Problem:
    """Noise-free matrix completion: M = A B^T with A (n1 x r), B (n2 x r)
    i.i.d. N(0,1); m distinct entries sampled uniformly without replacement;
    trace bound tau^2 = ||A||_F^2 + ||B||_F^2 (the trace of the planted
    feasible point [A; B][A; B]^T)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n1, r))
    B = rng.standard_normal((n2, r))
    total = n1 * n2
    assert m <= total
    if m > total // 4:
        lin = rng.choice(total, size=m, replace=False)
    else:
        lin = np.unique(rng.integers(0, total, size=int(m * 1.15) + 16))
        while lin.size < m:
            lin = np.unique(np.concatenate([lin, rng.integers(0, total, size=m)]))
        lin = rng.permutation(lin)[:m]
    lin.sort()
    ii, jj = lin // n2, lin % n2
    Mv = np.einsum("kr,kr->k", A[ii], B[jj])
    tau2 = float((A * A).sum() + (B * B).sum())
    p = mc_problem(n1, n2, ii, jj, Mv, tau2, name=f"mc{n1}x{n2}r{r}m{m}_s{seed}")
    p.meta.update({"A": A, "B": B, "r": r})
    return p


def phaselift_real(n: int, m: int, seed: int = 1) -> Problem:
    """Real-valued phase retrieval SDP (the real analogue of Section 5.4's
    complex formulation): min tr(X) s.t. a_l^T X a_l = (a_l^T x)^2, l = 1..m,
    with a_l i.i.d. N(0, I) and a planted x ~ N(0, I).  C = I (sparse
    diagonal), every constraint a rank-one low-rank term K = a_l, D = [1];
    trace bound tau^2 = ||x||^2, the trace of the planted point x x^T.  With
    m a few times n the SDP's solution is x x^T (exact recovery), so its value
    is ||x||^2."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    A = rng.standard_normal((m, n))
    i = np.arange(n)
    return Problem(name=f"phaselift_real_n{n}_m{m}_s{seed}", n=n, m=m, tau2=float(x @ x), row=i, col=i,
                   con=np.zeros(n, np.int64), val=np.ones(n), b=(A @ x) ** 2,
                   lr_con=list(range(1, m + 1)), lr_K=[A[l].reshape(n, 1) for l in range(m)],
                   lr_D=[np.ones((1, 1)) for _ in range(m)], meta={"kind": "phaselift", "x": x})


def cdp_masks(nc: int, L: int, rng: np.random.Generator) -> np.ndarray:
    """L octanary coded-diffraction masks of length nc: each entry is
    b1 * b2 with b1 uniform on {1, -1, i, -i} and b2 = sqrt(2)/2 with
    probability 0.8, sqrt(3) with probability 0.2 (the modulation of Candes,
    Li and Soltanolkotabi, "Phase retrieval from coded diffraction
    patterns", 2015; E|d|^2 = 1)."""
    b1 = np.array([1.0, -1.0, 1j, -1j])[rng.integers(0, 4, size=(L, nc))]
    b2 = np.where(rng.random((L, nc)) < 0.8, math.sqrt(2.0) / 2.0, math.sqrt(3.0))
    return b1 * b2


def phase_retrieval_cdp(nc: int, L: int = 12, seed: int = 1) -> Problem:
    """Complex phase retrieval from L coded diffraction patterns (Section
    5.4, eq. phase retrieval SDP; m = 12 n as in the paper's table):
    x in C^nc with i.i.d. standard complex Gaussian entries, measurements
    b_{l,k} = |(F (d_l * x))_k|^2 with F the unitary DFT.  The SDP
    min Tr X s.t. <a a^H, X> = b, X Hermitian PSD is stated on its real form
    (n = 2 nc, C = I as diagonal entries, see Problem.cdp_masks); the trace
    bound is ||x||^2.  With this many patterns the SDP recovers x x^H, so
    its optimum is ||x||^2."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(nc) + 1j * rng.standard_normal(nc)) / math.sqrt(2.0)
    d = cdp_masks(nc, L, rng)
    b = np.abs(np.fft.fft(d * x[None, :], axis=1, norm="ortho")) ** 2
    i = np.arange(2 * nc)
    return Problem(name=f"phase_cdp_n{nc}_L{L}_s{seed}", n=2 * nc, m=L * nc, tau2=float(np.vdot(x, x).real),
                   row=i, col=i, con=np.zeros(2 * nc, np.int64), val=np.ones(2 * nc), b=b.reshape(-1),
                   cdp_masks=d, meta={"kind": "phase_cdp", "x": x, "L": L})


def lowrank_constraints(n: int, m: int, seed: int = 1) -> Problem:
    """Random HSLR instance whose constraints mix the two parts of eq.
    HSLR-rep-body: the first 2m/3 constraints have sparse entries, the last
    2m/3 have a low-rank term K_l D_l K_l^T of rank 1 to 3 (the middle third
    both), one constraint two terms; the objective has a sparse part and a
    rank-2 low-rank term; b random (operator and eigen tests)."""
    rng = np.random.default_rng(seed)
    rows, cols, cons, vals = [], [], [], []
    for l in range(0, m):
        if l < 2 * m // 3:
            for _ in range(3):
                i, j = sorted(rng.integers(0, n, 2))
                rows.append(i); cols.append(j); cons.append(l + 1); vals.append(rng.standard_normal())
    for _ in range(2 * n):
        i, j = sorted(rng.integers(0, n, 2))
        rows.append(i); cols.append(j); cons.append(0); vals.append(rng.standard_normal())
    lr_con, lr_K, lr_D = [0], [rng.standard_normal((n, 2)) / np.sqrt(n)], [np.diag([1.0, -0.5])]
    for l in range(m // 3, m):
        r = int(rng.integers(1, 4))
        lr_con.append(l + 1)
        lr_K.append(rng.standard_normal((n, r)) / np.sqrt(n))
        D = rng.standard_normal((r, r))
        lr_D.append(D + D.T)
    lr_con.append(m)
    lr_K.append(rng.standard_normal((n, 1)) / np.sqrt(n))
    lr_D.append(np.array([[0.3]]))
    return Problem(name=f"lowrank_constraints_n{n}_m{m}_s{seed}", n=n, m=m, tau2=1.0, row=rows, col=cols, con=cons,
                   val=vals, b=0.01 * rng.standard_normal(m), lr_con=lr_con, lr_K=lr_K, lr_D=lr_D,
                   meta={"kind": "random"})


def served_stream_sizes(count: int = 4096, seed: int = 5, nmin: int = 100, nmax: int = 20_000):
    """Sizes of the served request stream: n log-uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(np.int64)


def served_request(k: int, n: int, seed: int = 5, avg_deg: float = 8.0) -> Problem:
    """Request k of the served stream: MaxCut SDP on G(n, avg_deg/(n-1)) with
    +-1 weights; its own generator is seeded from (seed, k)."""
    rng = np.random.default_rng([seed, k])
    i, j = er_edges(int(n), avg_deg / (n - 1), rng)
    w = pm1_weights(i.size, rng)
    return maxcut_problem(int(n), i, j, w, name=f"req{k}_n{n}")
