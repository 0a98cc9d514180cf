"""Write tests/golden/refs.json: FP64 oracle solves of the seeded workloads
the GPU solve tests compare against (eps = 1e-7, or a looser eps where the
oracle needs too long for 1e-7), with the a-posteriori objective bound
|pval - dval| + |p^T (A(X) - b)| of each solve.  Calls only oracle/ and the
instance generators.  Usage: python tests/golden/make_refs.py [case ...]"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sdp_instances as si  # noqa: E402
from sdp_instances.sdpa import random_sdpa_text, read_sdpa  # noqa: E402


def cases():
    yield "maxcut_er800_s1", si.maxcut_er_800(1), dict(rank_cap=16, rank_cap_truncate=True), 1e-7
    rng = np.random.default_rng(11)
    i, j = si.er_edges(400, 0.02, rng)
    yield "maxcut_pm1_er400", si.maxcut_problem(400, i, j, si.pm1_weights(i.size, rng), name="maxcut_pm1_er400"), {}, 1e-7
    yield "torus_pm1_20x20", si.maxcut_torus(20, 20, seed=3), {}, 1e-6
    rng = np.random.default_rng(12)
    i, j = si.er_edges(150, 0.06, rng)
    yield "theta_er150", si.theta_problem(150, i, j), {}, 1e-6
    yield "mc_60x90", si.mc_planted(60, 90, 2, 2500, seed=6), {}, 1e-7
    # the +-1 MaxCut requests of the serving pool test (ER, average degree 8)
    rng = np.random.default_rng(5)
    for n in (37, 150, 420, 1100):
        i, j = si.er_edges(n, 8.0 / (n - 1), rng)
        yield f"pool_er{n}", si.maxcut_problem(n, i, j, si.pm1_weights(i.size, rng)), {}, 1e-7
    # an SDPA problem with one dense constraint (split to a low-rank term)
    text, tr = random_sdpa_text(24, 8, seed=3)
    yield "sdpa_dense_24", read_sdpa(text, 3.0 * tr), {}, 1e-6


def main(only):
    path = os.path.join(os.path.dirname(__file__), "refs.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name, prob, kw, eps in cases():
        if only and name not in only:
            continue
        t = time.time()
        r = oracle.hallar(prob, si.gaussian_u0(prob.n, 7), oracle.Options(eps=eps, time_limit=1800, **kw))
        resid = oracle.a_tilde(prob, r.U)[1:] - prob.b
        bound = abs(r.pval - r.dval) + abs(float(r.p @ resid))
        out[name] = dict(pval=r.pval, dval=r.dval, status=r.status, rank=r.rank, eps=eps, opts=kw,
                         pinf=r.pinf, gap=r.gap, dinf=r.dinf, bound=bound, seconds=round(time.time() - t, 1))
        print(name, out[name], flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
