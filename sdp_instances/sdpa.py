"""Reader of SDPA sparse-format problems (".dat-s") into the HSLR form of
Section 3.2 (eq. HSLR-rep-body), with the dense split of Section 4.3: a
constraint matrix whose density d_l = nnz(A_l)/n^2 exceeds 0.1 is stored
densely -- here as the low-rank term K D K^T of its eigendecomposition (its
nonzero eigenpairs), which equals the dense matrix and runs on the low-rank
path of Algorithms 3 and 5 -- instead of as sparse entries.

SDPA's dual-form problem  max F_0 . Y  s.t.  F_l . Y = c_l (l = 1..m), Y PSD
is read as this library's  min C . X  s.t.  A_l . X = b_l  with C = -F_0,
A_l = F_l, b_l = c_l (so pval = -(SDPA objective)).  Several blocks are
placed on the diagonal of one n x n matrix (n = sum of the block sizes, a
negative size -k being a diagonal block of k entries): the data only touch
entries inside a block, so the optimum is unchanged.  HALLaR needs a trace
bound Tr X <= tau^2, which the format does not carry: the caller gives it.
"""
from __future__ import annotations

import re

import numpy as np

from . import Problem


def _tokens(text):
    """Numbers of the file in order: comment lines (starting with '"' or
    '*') are skipped, and so is any word that is not a number (the trailing
    '=mdim' style notes of the header lines, the braces and commas of a
    block-structure line)."""
    out = []
    for line in text.splitlines():
        s = line.strip()
        if not s or s[0] in "\"*":
            continue
        for w in re.split(r"[\s,{}()]+", s):
            try:
                float(w)
            except ValueError:
                continue
            out.append(w)
    return out


def read_sdpa(text: str, trace_bound: float, dense_threshold: float = 0.1, name: str = "sdpa") -> Problem:
    """Parse an SDPA sparse-format problem given as text."""
    tok = _tokens(text)
    pos = 0

    def nxt():
        nonlocal pos
        pos += 1
        return tok[pos - 1]

    m = int(nxt())
    nblocks = int(nxt())
    sizes = [int(float(nxt())) for _ in range(nblocks)]
    c = np.array([float(nxt()) for _ in range(m)])
    offs = np.cumsum([0] + [abs(s) for s in sizes])
    n = int(offs[-1])
    ents = {}  # matrix -> list of (i, j, value), upper triangle, summed on repeats
    while pos + 5 <= len(tok):
        mat, blk, i, j, v = int(nxt()), int(nxt()), int(nxt()), int(nxt()), float(nxt())
        if sizes[blk - 1] < 0 and i != j:
            raise ValueError("off-diagonal entry in a diagonal block")
        a, b = offs[blk - 1] + min(i, j) - 1, offs[blk - 1] + max(i, j) - 1
        ents.setdefault(mat, {})
        ents[mat][(a, b)] = ents[mat].get((a, b), 0.0) + v
    rows, cols, cons, vals = [], [], [], []
    lr_con, lr_K, lr_D = [], [], []
    for mat in range(0, m + 1):
        e = ents.get(mat, {})
        sign = -1.0 if mat == 0 else 1.0   # C = -F_0
        # density d_l = nnz(A_l) / n^2 over the full symmetric matrix (eq.
        # constraint matrix density)
        nnz = sum(1 if i == j else 2 for (i, j), v in e.items() if v != 0.0)
        if mat > 0 and nnz > dense_threshold * n * n:
            # dense constraint: its nonzero eigenpairs as a low-rank term
            A = np.zeros((n, n))
            for (i, j), v in e.items():
                A[i, j] = A[j, i] = v
            w, Q = np.linalg.eigh(A)
            keep = np.abs(w) > 1e-12 * max(1.0, float(np.abs(w).max(initial=0.0)))
            if keep.any():
                lr_con.append(mat)
                lr_K.append(Q[:, keep])
                lr_D.append(np.diag(w[keep]))
            continue
        for (i, j), v in e.items():
            rows.append(i)
            cols.append(j)
            cons.append(mat)
            vals.append(sign * v)
    return Problem(name=name, n=n, m=m, tau2=float(trace_bound), row=rows, col=cols, con=cons, val=vals, b=c,
                   lr_con=lr_con, lr_K=lr_K, lr_D=lr_D,
                   meta={"kind": "sdpa", "blocks": sizes, "dense_threshold": dense_threshold})


def write_sdpa(prob: Problem) -> str:
    """The problem in SDPA sparse format as one PSD block (sparse entries
    only; low-rank terms are written out densely), the inverse of read_sdpa
    for a one-block problem."""
    lines = [str(prob.m), "1", str(prob.n), " ".join(repr(float(v)) for v in prob.b)]
    acc = {}
    for i, j, l, v in zip(prob.row, prob.col, prob.con, prob.val):
        acc[(int(l), int(i), int(j))] = acc.get((int(l), int(i), int(j)), 0.0) + float(v)
    for l, K, D in zip(prob.lr_con, prob.lr_K, prob.lr_D):
        A = K @ D @ K.T
        for i in range(prob.n):
            for j in range(i, prob.n):
                if A[i, j] != 0.0:
                    acc[(int(l), i, j)] = acc.get((int(l), i, j), 0.0) + float(A[i, j])
    for (l, i, j), v in sorted(acc.items()):
        lines.append(f"{l} 1 {i + 1} {j + 1} {repr(-v if l == 0 else v)}")
    return "\n".join(lines) + "\n"


def random_sdpa_text(n: int, m: int, seed: int = 1):
    """A seeded SDPA text: min tr(Y) (F_0 = -I) subject to m - 1 sparse
    constraints of four random entries and one dense constraint (every upper
    entry N(0, 1)/n), with c = F(X_0) for a planted rank-2 PSD X_0 (so the
    problem is feasible).  Returns the text and tr(X_0)."""
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((n, 2))
    X0 = V @ V.T
    mats = [{(i, i): -1.0 for i in range(n)}]
    for l in range(1, m + 1):
        e = {}
        if l == m:
            for i in range(n):
                for j in range(i, n):
                    e[(i, j)] = rng.standard_normal() / n
        else:
            for _ in range(4):
                i, j = sorted(rng.integers(0, n, 2))
                e[(i, j)] = e.get((i, j), 0.0) + rng.standard_normal()
        mats.append(e)
    c = []
    for e in mats[1:]:
        c.append(sum((1.0 if i == j else 2.0) * v * X0[i, j] for (i, j), v in e.items()))
    out = [f"{m} =mdim", "1 =nblocks", f"{n}", " ".join(f"{v:.17g}" for v in c)]
    for l, e in enumerate(mats):
        for (i, j), v in sorted(e.items()):
            out.append(f"{l} 1 {i + 1} {j + 1} {v:.17g}")
    return "\n".join(out) + "\n", float(np.trace(X0))
