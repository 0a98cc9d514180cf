#!/usr/bin/env python3
"""Benchmark of the MI355X HALLaR hot path: SDP solves/s at 1e-5 relative
gap on one GPU, with the dominant kernel's achieved HBM bandwidth.

One step is one complete HALLaR solve (operators, ADAP-FISTA/ADAP-AIPP,
Lanczos, Frank-Wolfe, multiplier updates, relative termination) of a seeded
synthetic instance resident in HBM.  Workloads (--workload):
  mc      matrix completion, 1e5 x 1e5 rank 3, m = 1.2e7, FP64 (the
          paper's precision), rank cap 16 (default); then the same instance
          in FP32-mixed (--mixed-steps), reported beside it with its error
          against the FP64 solve
  torus   MaxCut SDP, 1000 x 1000 torus (n = 1e6), +-1 weights, FP32-mixed,
          rank cap 32 (does not reach 1e-5 within the limits: its solution
          rank grows with n far beyond 32)
  er800   MaxCut SDP, G(800, 0.02), unit weights, FP64, rank cap 16
  theta   Lovasz theta SDP, G(5e4, avg deg 10), FP32-mixed, rank cap 64
  hamming Lovasz theta SDP of the Hamming graph H(20, 2) (n = 2^20,
          m = 10,485,760 edge constraints), FP64; theta = n/2 exactly
  phase   complex phase retrieval, n = 1e5 unknowns, 12 coded diffraction
          patterns (m = 1.2e6), FFT operators, FP64; optimum ||x||^2
  served  stream of MaxCut requests (n log-uniform in [100, 2e4], deg 8,
          +-1 weights) through the continuous-batching pool; reports p50/p99
  ops     operator-level timing (SDDMM and SpMM entry points, --ops-instance
          mc or torus) with a 1 GiB copy for HBM counter calibration
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HAMMING_D = 20


def workload(name):
    import sdp_instances as si
    from paper_2505_13719_amd import hallar as H
    if name == "torus":
        return si.maxcut_torus(1000, 1000, seed=2), H.FP32_MIXED, dict(rank_cap=32, rank_cap_truncate=1), \
            {"workload": "maxcut_torus_1000x1000_pm1", "n": 10 ** 6, "edges": 2 * 10 ** 6, "rank_cap": 32}
    if name == "er800":
        return si.maxcut_er_800(1), H.FP64, dict(rank_cap=16, rank_cap_truncate=1), \
            {"workload": "maxcut_er_800_p0.02", "n": 800, "rank_cap": 16}
    if name == "theta":
        return si.theta_er(50_000, 10.0, seed=3), H.FP32_MIXED, dict(rank_cap=64), \
            {"workload": "theta_er_50000_deg10", "n": 50_000, "rank_cap": 64}
    if name == "hamming":
        # Table tab:reduced_hamming_graphs: H(d, 2), theta = n/2 (d = 20 by
        # default; the table goes to d = 23)
        d = HAMMING_D
        n = 1 << d
        prob = si.theta_problem(n, *si.hypercube_edges(d), name=f"hamming_{d}_2")
        prob.meta["optimum"] = -n / 2
        return prob, H.FP64, {}, {"workload": f"theta_hamming_H({d},2)", "n": n, "m": int(prob.m)}
    if name == "phase":
        # complex phase retrieval from 12 coded diffraction patterns (Section
        # 5.4, the table's n = 100,000, m = 1,200,000 row), on the real form;
        # exact recovery: the optimum is ||x||^2
        nc = 100_000
        prob = si.phase_retrieval_cdp(nc, 12, seed=1)
        prob.meta["optimum"] = prob.tau2
        return prob, H.FP64, {}, {"workload": "phase_retrieval_cdp_n1e5_L12", "n_complex": nc, "n": 2 * nc,
                                  "m": 12 * nc}
    if name == "lowrank":
        # low-rank constraint terms (Section 3.2, eq. HSLR-rep-body) with
        # about 3900 columns of K in all on n = 1e5 rows: the dense
        # contraction K^T U of Algorithms 3 and 5 dominates the operators
        prob = si.lowrank_constraints(100_000, 2900, seed=7)
        rk = sum(K.shape[1] for l, K in zip(prob.lr_con, prob.lr_K) if l > 0)
        return prob, H.FP64, {}, {"workload": "lowrank_constraints_n1e5_m2900", "n": prob.n, "m": prob.m, "rk": rk}
    if name == "mc":
        n1 = n2 = 100_000
        return si.mc_planted(n1, n2, 3, 20 * 3 * (n1 + n2), seed=4), H.FP64, dict(rank_cap=16), \
            {"workload": "matrix_completion_1e5x1e5_r3_m1.2e7", "n": n1 + n2, "m": 20 * 3 * (n1 + n2)}
    raise ValueError(name)


PROFILE_TAG = {"mc": "mc_1e5x1e5_r3", "torus": "torus_1000x1000_pm1", "er800": "maxcut_er800", "phase": "phase_cdp_1e5",
               "theta": "theta_er50000", "served": "served_maxcut"}
CLASS_KERNEL = {"sddmm": "k_sddmm<", "spmm": "k_spmm<", "lanczos_spmv": "k_lz_spmv", "sddmm_spmm": "k_trial_fused<"}


def counted_traffic(workload_name, cls, prec=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (two rocprofv3 --pmc passes, calibrated on a 1 GiB copy), or None
    when there is none or the kernels changed since it was taken.  prec
    (0 FP64, 1 FP32-mixed) selects the kernel's instantiation."""
    import hashlib
    tag = PROFILE_TAG.get(workload_name)
    if tag is None or cls not in CLASS_KERNEL:
        return None
    if prec is not None:
        tag += "_fp64" if prec == 0 else "_fp32"
    path = os.path.join(ROOT, "profiles", tag + "_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = os.path.join(ROOT, "paper_2505_13719_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if "kernels.hip sha256[:16] = " + sha not in text:
        return None
    # every instantiation of the class's kernel in this precision, weighted
    # by its dispatches (the profile class aggregates them the same way)
    pat = CLASS_KERNEL[cls] + ("" if prec is None else ("double" if prec == 0 else "float"))
    tot, cnt = 0.0, 0
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch[") and pat in line:
            rhs = line.split("] = ", 1)[1].split()
            n = int(rhs[1].split("=")[1]) if len(rhs) > 1 else 1
            tot += float(rhs[0]) * n
            cnt += n
    return round(tot / cnt) if cnt else None


def roofline_from_profile(prof):
    """Dominant kernel class by time among the memory-streaming classes."""
    cands = {k: v for k, v in prof.items() if v["bytes"] > 0 and v["ms"] > 0}
    if not cands:
        return None, {}
    dom = max(cands, key=lambda k: cands[k]["ms"])
    v = cands[dom]
    achieved = v["bytes"] / (v["ms"] * 1e-3) / 1e9
    table = {k: dict(ms=round(x["ms"], 3), launches=x["launches"],
                     gbs=round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1) if x["ms"] > 0 and x["bytes"] > 0 else None,
                     us_per_launch=round(1e3 * x["ms"] / x["launches"], 2) if x["launches"] else None)
             for k, x in prof.items()}
    return dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                bytes_per_launch=v["bytes"] / max(v["launches"], 1),
                us_per_launch=1e3 * v["ms"] / max(v["launches"], 1)), table


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:  # pragma: no cover
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    return model, nproc


def cpu_baseline(prob, res, budget_s=20.0, c0_solve=False):
    """The FP64 oracle timed on the host on a bounded sample of the same
    instance: its SDDMM (A~(UU^T)), SpMM ((C + A*(y))U) and Lanczos product
    (with full reorthogonalisation) at the GPU solve's final rank, each timed
    on its own, then scaled by the GPU solve's operation counts (a FISTA trial
    is 2 SDDMM + 1 SpMM).  `cores` is the average number of threads the
    sample kept busy (process CPU time / wall time).  With c0_solve, also one
    complete oracle solve of the 800-vertex MaxCut SDP (eps = 1e-5; about
    two minutes on the host, so not in the default run)."""
    import numpy as np

    import oracle
    import sdp_instances as si
    model, nproc = host_cpu()
    r = max(int(res["rank"]), 1)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((prob.n, r)) / math.sqrt(prob.n * r) * math.sqrt(prob.tau2)
    ptil = np.concatenate([[1.0], rng.standard_normal(prob.m) * 1e-3])
    cpu0, wall0 = time.process_time(), time.perf_counter()

    def timed(fn, share):
        t0, k = time.perf_counter(), 0
        while True:
            fn()
            k += 1
            if time.perf_counter() - t0 > share or k >= 20:
                return (time.perf_counter() - t0) / k, k

    t_sddmm, k1 = timed(lambda: oracle.a_tilde(prob, U), budget_s / 3)
    t_spmm, k2 = timed(lambda: oracle.adjoint_apply(prob, ptil, U), budget_s / 3)
    if prob.lr_con or getattr(prob, "cdp_masks", None) is not None:
        mv = lambda x: oracle.adjoint_apply(prob, ptil, x)  # noqa: E731
    else:
        M = oracle.adjoint_sparse(prob, ptil)
        mv = lambda x: M @ x  # noqa: E731
    t1 = time.perf_counter()
    kmax = 32 if prob.n > 100_000 else 64
    _, _, info = oracle.min_eig(mv, prob.n, rng.standard_normal(prob.n), tol=1e-30, kmax=kmax, max_restarts=1)
    t_mv = (time.perf_counter() - t1) / max(info["iters"], 1)
    cores = (time.process_time() - cpu0) / max(time.perf_counter() - wall0, 1e-9)
    t_trial = 2 * t_sddmm + t_spmm
    est = res["n_fista_trials"] * t_trial + res["n_matvec"] * t_mv
    out = dict(value=round(1.0 / est, 8), unit="solves/s", cores=round(cores, 1), kind="oracle",
               sample=f"{k1} SDDMM and {k2} SpMM calls (rank {r}) and {info['iters']} Lanczos products with full "
                      f"reorthogonalisation on the full instance; a FISTA trial (2 SDDMM + 1 SpMM) costs "
                      f"{t_trial:.3f} s, scaled by the GPU solve's {res['n_fista_trials']} trials and "
                      f"{res['n_matvec']} products (estimated oracle solve {est:.0f} s)",
               per_op_ms={"sddmm": round(1e3 * t_sddmm, 1), "spmm": round(1e3 * t_spmm, 1),
                          "lanczos_product": round(1e3 * t_mv, 2)},
               est_seconds=round(est, 1), cpu_model=model, nproc=nproc)
    if c0_solve:
        c0 = si.maxcut_er_800(1)
        t2 = time.perf_counter()
        rc0 = oracle.hallar(c0, si.gaussian_u0(c0.n, 7),
                            oracle.Options(eps=1e-5, rank_cap=16, rank_cap_truncate=True, time_limit=120.0))
        out["maxcut_er800_oracle_solve"] = {"seconds": round(time.perf_counter() - t2, 2), "status": rc0.status,
                                            "pval": rc0.pval, "solves_per_s": round(1.0 / (time.perf_counter() - t2), 4)}
    return out


def copy_peak_gbs(reps=5):
    """Achievable HBM rate on this GPU: a plain 1 GiB device copy (read + write),
    timed with events after a warm-up copy."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return round(2 * (1 << 30) / sec / 1e9, 1)


def timed_solves(prob, prec, kw, steps, warmup, args, label):
    """Create a handle, run `warmup` untimed and `steps` timed solves from the
    same U0 (instance and U0 resident in HBM), return the wall time of the
    timed ones, the last result, the per-class profile and the schedule."""
    import torch

    import sdp_instances as si
    from paper_2505_13719_amd import hallar as H

    dev = torch.device("cuda:0")
    opts = H.options(eps=1e-5, profile=args.profile, time_limit=3000.0, verbose=args.verbose, autotune=args.autotune,
                     graphs=args.graphs, **kw)
    t_build = time.perf_counter()
    h = H.hallar_create(prob, prec, opts)
    t_build = time.perf_counter() - t_build
    schedule = dict(zip(("min_rows", "ent_cap", "ntiles"), H.hallar_schedule(h)))
    U0 = torch.tensor(si.gaussian_u0(prob.n, 7), device=dev)
    res = None
    for _ in range(warmup):
        res = H.hallar_solve(h, U0)
        print(f"[bench] {label} warmup solve: {res['status']} {res['seconds']:.2f}s", file=sys.stderr, flush=True)
    H.hallar_profile(h, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        res = H.hallar_solve(h, U0)
        print(f"[bench] {label} step {k}: {res['status']} pval={res['pval']:.9g} gap={res['gap']:.2e} "
              f"rank={res['rank']} {res['seconds']:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = H.hallar_profile(h)
    H.hallar_destroy(h)
    return dt, res, prof, schedule, t_build


def closed_form_optimum(prob):
    """The SDP's optimum where a closed form is known: noise-free matrix
    completion with exact recovery (||A B^T||_* from QR factors and an r x r
    SVD), and theta of a perfect graph (n/2 for the bipartite H(d, 2)).  None
    otherwise."""
    import numpy as np
    if "optimum" in prob.meta:
        return float(prob.meta["optimum"])
    if "A" not in prob.meta:
        return None
    _, ra = np.linalg.qr(prob.meta["A"])
    _, rb = np.linalg.qr(prob.meta["B"])
    return float(np.linalg.svd(ra @ rb.T, compute_uv=False).sum())


def bench_solve(args):
    from paper_2505_13719_amd import hallar as H

    prob, prec, kw, cfg = workload(args.workload)
    if args.precision:
        prec = H.FP64 if args.precision == "fp64" else H.FP32_MIXED
    dt, res, prof, schedule, t_build = timed_solves(prob, prec, kw, args.steps, args.warmup, args,
                                                    "fp64" if prec == H.FP64 else "fp32_mixed")
    roof, table = roofline_from_profile(prof)
    if roof:
        roof["traffic"] = counted_traffic(args.workload, roof["kernel"], prec)
        # the same achieved rate against what a plain copy reaches here
        roof["copy_gbs"] = copy_peak_gbs()
        roof["frac_of_copy"] = round(roof["achieved"] / roof["copy_gbs"], 4)
    opt = closed_form_optimum(prob)
    out = {
        "metric": "SDP solves/s at 1e-5 rel gap",
        "value": round(args.steps / dt, 6),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == H.FP64 else "f32+f64",
        "data": "synthetic",
        "config": dict(cfg, precision="fp64" if prec == H.FP64 else "fp32_mixed", eps=1e-5),
        "solve": {k: res[k] for k in ("status", "pval", "dval", "pinf", "gap", "dinf", "obj_bound", "rank",
                                      "outer_iters", "n_fista_trials", "n_matvec", "n_hlr_iters", "n_eig_calls",
                                      "n_rounds", "n_truncations")},
        "roofline": roof,
        "kernels": table,
        "create_s": round(t_build, 2),
        "schedule": dict(schedule, autotuned=bool(args.autotune)),
    }
    if opt is not None:
        out["solve"]["closed_form_optimum"] = opt
        out["solve"]["objective_rel_error"] = abs(res["pval"] - opt) / (1.0 + abs(opt))
    if prec == H.FP64 and args.mixed_steps > 0:
        # the FP32-mixed systems form on the same instance, timed after the
        # headline steps, with its error against the FP64 solve
        dt32, r32, prof32, _, _ = timed_solves(prob, H.FP32_MIXED, kw, args.mixed_steps, 1, args, "fp32_mixed")
        roof32, _ = roofline_from_profile(prof32)
        v32 = args.mixed_steps / dt32
        mixed = {"solves_per_s": round(v32, 6), "steps": args.mixed_steps,
                 "speedup_vs_fp64": round(v32 / out["value"], 3), "status": r32["status"], "pval": r32["pval"],
                 "gap": r32["gap"], "pinf": r32["pinf"], "obj_bound": r32["obj_bound"],
                 "rel_diff_vs_fp64": abs(r32["pval"] - res["pval"]) / (1.0 + abs(res["pval"])),
                 "dominant_kernel": roof32 and {k: roof32[k] for k in ("kernel", "achieved", "frac", "us_per_launch")}}
        if opt is not None:
            mixed["objective_rel_error"] = abs(r32["pval"] - opt) / (1.0 + abs(opt))
        out["fp32_mixed"] = mixed
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, res, budget_s=args.cpu_budget, c0_solve=args.cpu_c0_solve)
    if args.served_sample > 0:
        # the serving form on the first requests of the served MaxCut stream
        # (all arriving at t = 0), beside the plain FP64 solver on the same
        # requests; not part of the headline value
        sv = bench_served(args, nreq=args.served_sample, fifo_sample=args.served_sample)
        out["served"] = dict(sv["served"], solves_per_s=sv["value"], requests=args.served_sample,
                             workload=sv["config"]["workload"], n_range=sv["config"]["n_range"],
                             fifo_fp64=sv["fifo_fp64"])
    return out


def bench_served(args, nreq=None, fifo_sample=None):
    """The served MaxCut stream through the continuous-batching pool (FP32 +
    FP64), then the plain per-instance FP64 solver FIFO on the first
    fifo_sample requests of the same stream, with each served result's
    objective error against that FP64 solve of the same request."""
    import numpy as np
    import torch

    import sdp_instances as si
    from paper_2505_13719_amd import hallar as H

    nreq = args.served_requests if nreq is None else nreq
    fifo_sample = args.fifo_sample if fifo_sample is None else fifo_sample
    sizes = si.served_stream_sizes(4096, seed=5)[:nreq]
    rng = np.random.default_rng(6)
    t_gen = time.perf_counter()
    reqs = [si.served_request(k, int(n), seed=5) for k, n in enumerate(sizes)]
    U0s = [si.gaussian_u0(int(n), 1000 + k) for k, n in enumerate(sizes)]
    t_gen = time.perf_counter() - t_gen
    # the larger requests (n ~ 1e4 - 2e4) pass the library's 63-column limit
    # on the way to their optimum: they keep the largest directions there
    # (counted in n_truncations) and the final certificate judges the result
    opts = H.options(eps=1e-5, profile=args.profile, verbose=args.verbose, graphs=args.graphs, rank_cap_truncate=1)
    rate = args.rate
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq)) if rate > 0 else np.zeros(nreq)
    pool = H.hallar_pool_create(int(args.budget_gb * (1 << 30)), args.max_active, H.FP32_MIXED, opts)
    done = {}
    nxt = 0
    max_active = 0
    torch.cuda.synchronize()
    print(f"[bench] served: {nreq} requests generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    t_print = 0.0
    while len(done) < nreq:
        now = time.perf_counter() - t0
        if now - t_print > 5.0:
            t_print = now
            print(f"[bench] served t={now:.1f}s admitted={nxt} done={len(done)} active={max_active}",
                  file=sys.stderr, flush=True)
        while nxt < nreq and arrivals[nxt] <= now:
            st = H.hallar_pool_admit(pool, reqs[nxt], nxt, U0=U0s[nxt])
            if st != "ok":
                break
            nxt += 1
        act = H.hallar_pool_step(pool, 1)
        max_active = max(max_active, act)
        tnow = time.perf_counter() - t0
        for t, r in H.hallar_pool_poll(pool):
            done[t] = (tnow, r)
        if act == 0 and nxt < nreq and arrivals[nxt] > tnow:
            time.sleep(min(arrivals[nxt] - tnow, 0.01))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = H.hallar_pool_profile(pool)
    H.hallar_pool_destroy(pool)
    lat = np.array([done[k][0] - arrivals[k] for k in range(nreq)])
    ok = sum(1 for k in range(nreq) if done[k][1]["status"] == "ok")
    statuses = {}
    for k in range(nreq):
        st_k = done[k][1]["status"]
        statuses[st_k] = statuses.get(st_k, 0) + 1
        if st_k != "ok":
            r_k = done[k][1]
            print(f"[bench] request {k} n={reqs[k].n}: {st_k} rank={r_k['rank']} outer={r_k['outer_iters']} "
                  f"gap={r_k['gap']:.2e} pinf={r_k['pinf']:.2e} obj_bound={r_k['obj_bound']:.3g} "
                  f"pval={r_k['pval']:.9g}", file=sys.stderr, flush=True)
    first = float(arrivals.min())
    last = max(v[0] for v in done.values())
    roof, table = roofline_from_profile(prof)
    if roof:
        roof["traffic"] = counted_traffic("served", roof["kernel"])
    fifo = None
    if fifo_sample > 0:
        # the plain per-instance FP64 solver on the first requests of the same
        # stream, one at a time on the same stream
        k = min(fifo_sample, nreq)
        ok64 = 0
        errs = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for q in range(k):
            h = H.hallar_create(reqs[q], H.FP64, H.options(eps=1e-5, rank_cap_truncate=1))
            r = H.hallar_solve(h, torch.tensor(U0s[q], device="cuda:0"))
            H.hallar_destroy(h)
            ok64 += r["status"] == "ok"
            errs.append(abs(done[q][1]["pval"] - r["pval"]) / (1.0 + abs(r["pval"])))
            print(f"[bench] fifo fp64 {q + 1}/{k}: n={reqs[q].n} {r['status']} {r['seconds']:.2f}s "
                  f"served-vs-fp64 {errs[-1]:.2e}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_fifo = time.perf_counter() - t1
        fifo = {"requests": k, "solves_per_s": round(k / t_fifo, 4), "converged": ok64,
                "served_rel_error_vs_fp64": {"max": float(max(errs)), "median": float(np.median(errs))}}
    out = {
        "metric": "SDP solves/s at 1e-5 rel gap",
        "value": round(nreq / (last - first), 4),
        "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * dt, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "served_maxcut_stream", "requests": nreq, "rate_per_s": rate,
                   "n_range": [int(sizes.min()), int(sizes.max())], "budget_gb": args.budget_gb,
                   "max_active": args.max_active},
        "served": {"p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
                   "converged": ok, "statuses": statuses, "max_active": max_active, "gen_s": round(t_gen, 1),
                   "truncated_requests": sum(1 for k in range(nreq) if done[k][1]["n_truncations"] > 0)},
        "fifo_fp64": fifo,
        "roofline": roof,
        "kernels": table,
    }
    return out


def bench_ops(args):
    """Operator-level timing on the instance of --ops-instance (the workload's
    precision unless --precision; r = 4 for matrix completion, 32 for the
    torus, both column buckets, so U and W are used in place): hallar_eval_AUUt (SDDMM +
    AL epilogue) and hallar_adjoint_spmm (SpMM), each called --steps times on a
    random U, plus a plain 1 GiB device copy (the calibration kernel for the
    HBM byte counters)."""
    import numpy as np
    import torch

    from paper_2505_13719_amd import hallar as H

    prob, prec, kw, cfg = workload(args.ops_instance)
    if args.precision:
        prec = H.FP64 if args.precision == "fp64" else H.FP32_MIXED
    dt = torch.float64 if prec == H.FP64 else torch.float32
    dev = torch.device("cuda:0")
    r = 32 if args.ops_instance == "torus" else 4
    h = H.hallar_create(prob, prec, H.options(eps=1e-5, profile=1, **kw))
    g = torch.Generator(device="cpu").manual_seed(0)
    U = (torch.randn((prob.n, r), generator=g, dtype=dt) / math.sqrt(r)).to(dev)
    W = torch.empty_like(U)
    T = torch.empty(prob.m + 1, dtype=torch.float64, device=dev)
    p = torch.tensor(np.random.default_rng(1).standard_normal(prob.m), device=dev)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(2):
        H.hallar_eval_AUUt(h, U, T)
        H.hallar_adjoint_spmm(h, p, U, W)
        dst.copy_(src)
    torch.cuda.synchronize()
    out = {}
    for name, fn in (("eval_AUUt", lambda: H.hallar_eval_AUUt(h, U, T)),
                     ("adjoint_spmm", lambda: H.hallar_adjoint_spmm(h, p, U, W)),
                     ("copy_1GiB", lambda: dst.copy_(src))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1) * 1e3 / args.steps, 2)
        print(f"[bench] {name}: {out[name]} us/call", file=sys.stderr, flush=True)
    H.hallar_destroy(h)
    res = {"metric": "operator us/call", "config": dict(cfg, r=r, precision="fp64" if prec == H.FP64 else "fp32_mixed"),
           "us_per_call": out,
           "copy_gbs": round(2 * (1 << 30) / (out["copy_1GiB"] * 1e-6) / 1e9, 1)}
    if "rk" in cfg:
        # K (n x rk, operator type) read once per evaluation and once per
        # adjoint: its rate against the HBM peak
        kb = prob.n * cfg["rk"] * (8 if prec == H.FP64 else 4)
        res["K_bytes"] = kb
        res["K_gbs"] = {k: round(kb / (out[k] * 1e-6) / 1e9, 1) for k in ("eval_AUUt", "adjoint_spmm")}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hamming-d", type=int, default=20, help="d of H(d, 2) for --workload hamming (10..23)")
    ap.add_argument("--workload", default="mc",
                    choices=["torus", "er800", "theta", "mc", "hamming", "phase", "served", "ops"])
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", type=int, default=0, help="solver progress on stderr (1: outer, 2: HLR)")
    ap.add_argument("--profile", type=int, default=2, choices=[0, 1, 2],
                    help="HIP-event timing inside the timed solves: 2 = the sparse kernel classes only (default, "
                         "least overhead), 1 = every class, 0 = none (repeating rounds then replay captured graphs)")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1], help="opts.graphs (used when --profile 0)")
    ap.add_argument("--ops-instance", default="mc", choices=["mc", "torus", "lowrank"], help="instance of --workload ops")
    ap.add_argument("--autotune", type=int, default=0, help="1: tune the tile schedule at create (timed outside the steps)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-c0-solve", action="store_true",
                    help="cpu_baseline: also time one complete oracle solve of the 800-vertex MaxCut SDP")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="FP64 runs: also time this many FP32-mixed solves of the same instance (0: none)")
    ap.add_argument("--served-requests", type=int, default=4096)
    ap.add_argument("--served-sample", type=int, default=32,
                    help="solve workloads: also serve this many requests of the served stream at t = 0 and solve "
                         "them FIFO with the plain FP64 solver (0: none)")
    ap.add_argument("--rate", type=float, default=0.0, help="Poisson arrivals per second (0: all at t = 0)")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--max-active", type=int, default=1024)
    ap.add_argument("--fifo-sample", type=int, default=32,
                    help="served: also solve this many requests one at a time with the plain FP64 solver")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    global HAMMING_D
    if not 10 <= args.hamming_d <= 23:
        print("--hamming-d takes 10..23 (the graphs of the table)", file=sys.stderr)
        sys.exit(2)
    HAMMING_D = args.hamming_d
    if args.workload == "ops":
        out = bench_ops(args)
    else:
        out = bench_served(args) if args.workload == "served" else bench_solve(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
