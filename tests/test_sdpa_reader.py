"""The SDPA sparse-format reader and the dense split (Section 4.3: a
constraint denser than d_l > 0.1 stored as a low-rank term from its
eigendecomposition).

* A two-by-two problem written by hand: min tr(Y) s.t. Y_12 = 1, Y PSD has
  the optimum 2 (Y_11 Y_22 >= 1 and the AM-GM bound); the oracle solve of
  the parsed problem reaches it.
* Blocks placed on the diagonal: a problem written as two blocks (one of
  them a diagonal block) and the same data written as one block give the
  same A~(UU^T) and A~*(p~)U.
* The dense split changes only the storage: the split and the unsplit
  readings of the same text give the same operators to rounding.
* write_sdpa / read_sdpa round-trip the generators' problems.
"""
import numpy as np

import oracle
import sdp_instances as si
from sdp_instances.sdpa import read_sdpa, write_sdpa

# max -tr(Y) s.t. Y_12 = 1 in SDPA's dual form (F_0 = -I, F_1 with 1/2 off
# the diagonal so that F_1 . Y = Y_12)
TWO_BY_TWO = """\
"a two-by-two example"
1 =mdim
1 =nblocks
2
1.0
0 1 1 1 -1.0
0 1 2 2 -1.0
1 1 1 2 0.5
"""


def _ops_close(p, q, seed=0, r=3, tol=1e-12):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((p.n, r))
    pt = rng.standard_normal(p.m + 1)
    Tp, Tq = oracle.a_tilde(p, U), oracle.a_tilde(q, U)
    assert np.abs(Tp - Tq).max() <= tol * (1.0 + np.abs(Tp).max())
    Wp, Wq = oracle.adjoint_apply(p, pt, U), oracle.adjoint_apply(q, pt, U)
    assert np.abs(Wp - Wq).max() <= tol * (1.0 + np.abs(Wp).max())


def test_two_by_two_optimum():
    prob = read_sdpa(TWO_BY_TWO, trace_bound=3.0)
    assert (prob.n, prob.m, list(prob.b)) == (2, 1, [1.0])
    # C = -F_0 = I, A_1 = F_1
    # (one entry of three is above the density threshold: A_1 is stored as
    # its low-rank eigendecomposition)
    assert prob.lr_con == [1]
    C = oracle.adjoint_apply(prob, np.array([1.0, 0.0]), np.eye(2))
    A1 = oracle.adjoint_apply(prob, np.array([0.0, 1.0]), np.eye(2))
    assert np.array_equal(C, np.eye(2)) and np.abs(A1 - [[0.0, 0.5], [0.5, 0.0]]).max() <= 1e-15
    res = oracle.hallar(prob, si.gaussian_u0(prob.n, 3), oracle.Options(eps=1e-7))
    assert res.status == "ok"
    assert abs(res.pval - 2.0) <= 1e-6 * 3.0


def test_blocks_on_the_diagonal():
    two_blocks = """2 2
3 -2
1.0 2.0
0 1 1 1 1.0
0 1 1 3 0.25
0 2 1 1 -2.0
1 1 2 3 0.5
1 2 2 2 1.5
2 1 3 3 1.0
2 2 1 1 4.0
"""
    one_block = """2 1
5
1.0 2.0
0 1 1 1 1.0
0 1 1 3 0.25
0 1 4 4 -2.0
1 1 2 3 0.5
1 1 5 5 1.5
2 1 3 3 1.0
2 1 4 4 4.0
"""
    p, q = read_sdpa(two_blocks, 10.0), read_sdpa(one_block, 10.0)
    assert p.n == q.n == 5 and p.meta["blocks"] == [3, -2]
    _ops_close(p, q)


def _dense_text(n, m, seed):
    """One sparse constraint set plus a dense constraint (every entry)."""
    rng = np.random.default_rng(seed)
    lines = [str(m), "1", str(n), " ".join(f"{v:.17g}" for v in rng.standard_normal(m))]
    for i in range(n):
        lines.append(f"0 1 {i + 1} {i + 1} 1.0")
    for l in range(1, m):
        i, j = sorted(rng.integers(1, n + 1, 2))
        lines.append(f"{l} 1 {i} {j} {rng.standard_normal():.17g}")
    for i in range(1, n + 1):              # constraint m: dense, rank n
        for j in range(i, n + 1):
            lines.append(f"{m} 1 {i} {j} {rng.standard_normal():.17g}")
    return "\n".join(lines) + "\n"


def test_dense_split_same_operators():
    text = _dense_text(12, 5, seed=4)
    split = read_sdpa(text, 4.0, dense_threshold=0.1)
    plain = read_sdpa(text, 4.0, dense_threshold=2.0)   # never split
    assert split.lr_con == [5] and plain.lr_con == []
    assert split.lr_K[0].shape[1] == 12                  # a generic dense matrix keeps every eigenpair
    assert not (split.con == 5).any()
    _ops_close(split, plain, tol=1e-12)


def test_dense_split_keeps_rank():
    # a dense rank-two constraint v v^T - w w^T stays rank two after the split
    rng = np.random.default_rng(8)
    n = 9
    v, w = rng.standard_normal(n), rng.standard_normal(n)
    A = np.outer(v, v) - np.outer(w, w)
    lines = ["1", "1", str(n), "0.5"] + [f"0 1 {i + 1} {i + 1} 1.0" for i in range(n)]
    lines += [f"1 1 {i + 1} {j + 1} {A[i, j]:.17g}" for i in range(n) for j in range(i, n)]
    prob = read_sdpa("\n".join(lines) + "\n", 2.0)
    assert prob.lr_con == [1] and prob.lr_K[0].shape[1] == 2
    K, D = prob.lr_K[0], prob.lr_D[0]
    assert np.abs(K @ D @ K.T - A).max() <= 1e-12 * np.abs(A).max()


def test_round_trip_generators():
    rng = np.random.default_rng(2)
    i, j = si.er_edges(30, 0.2, rng)
    for prob in (si.maxcut_problem(30, i, j, si.pm1_weights(i.size, rng)), si.theta_problem(10, *si.petersen_edges()),
                 si.lowrank_constraints(20, 9, seed=3)):
        back = read_sdpa(write_sdpa(prob), prob.tau2, dense_threshold=2.0)
        _ops_close(prob, back, tol=1e-12)
