"""The host-side problem preprocessing (descriptor validation, pair and
entry lists, tiles, low-rank terms, coded-diffraction masks, the Jacobi
eigensolver) built with the host address and undefined-behaviour
sanitizers (device code unaffected) and run on valid and invalid
descriptors of every family: no sanitizer report, and the same structure as
the library's own build reports through hallar_inspect."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import sdp_instances as si
from paper_2505_13719_amd import hallar as H
from sdp_instances.sdpa import random_sdpa_text, read_sdpa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker():
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp(prefix="hallar_host_check_")
    exe = os.path.join(d, "host_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I" + os.path.join(ROOT, "include"), "-x", "hip", os.path.join(ROOT, "tests", "host_check.cpp"),
           os.path.join(ROOT, "paper_2505_13719_amd", "csrc", "problem.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    yield d, exe
    shutil.rmtree(d, ignore_errors=True)


def _write(path, prob, n=None, m=None):
    n = prob.n if n is None else n
    m = prob.m if m is None else m
    with open(path, "wb") as f:
        np.array([n, m], np.int64).tofile(f)
        np.array([prob.tau2], np.float64).tofile(f)
        np.array([prob.row.size], np.int64).tofile(f)
        for a in (prob.row, prob.col, prob.con):
            np.asarray(a, np.int32).tofile(f)
        np.asarray(prob.val, np.float64).tofile(f)
        np.asarray(prob.b, np.float64)[:m].tofile(f)
        nl = len(prob.lr_con)
        np.array([nl], np.int32).tofile(f)
        np.asarray(prob.lr_con, np.int32).tofile(f)
        np.asarray([K.shape[1] for K in prob.lr_K], np.int32).tofile(f)
        Ks = [np.ascontiguousarray(K, np.float64).reshape(-1) for K in prob.lr_K]
        Ds = [np.ascontiguousarray(D, np.float64).reshape(-1) for D in prob.lr_D]
        np.cumsum([0] + [k.size for k in Ks])[:nl].astype(np.int64).tofile(f)
        np.cumsum([0] + [x.size for x in Ds])[:nl].astype(np.int64).tofile(f)
        K = np.concatenate(Ks) if Ks else np.zeros(0)
        D = np.concatenate(Ds) if Ds else np.zeros(0)
        np.array([K.size, D.size], np.int64).tofile(f)
        K.tofile(f)
        D.tofile(f)
        masks = getattr(prob, "cdp_masks", None)
        mv = np.zeros(0) if masks is None else np.ascontiguousarray(masks, np.complex128).view(np.float64).reshape(-1)
        np.array([0 if masks is None else masks.shape[0]], np.int32).tofile(f)
        np.array([mv.size], np.int64).tofile(f)
        mv.tofile(f)


def _valid():
    rng = np.random.default_rng(3)
    i, j = si.er_edges(60, 0.1, rng)
    text, tr = random_sdpa_text(20, 6, seed=2)
    return [si.maxcut_problem(60, i, j, si.pm1_weights(i.size, rng)), si.theta_problem(10, *si.petersen_edges()),
            si.mc_planted(30, 40, 2, 600, seed=1), si.lowrank_constraints(50, 15, seed=4),
            si.phaselift_real(12, 40, seed=2), si.phase_retrieval_cdp(16, 3, seed=1), read_sdpa(text, 2.0 * tr),
            si.random_hslr(40, 20, 1), si.random_hslr(40, 20, 2, lowrank_nonobjective=True)]


def test_host_preprocessing_sanitized(checker):
    d, exe = checker
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probs = _valid()
    paths = []
    for k, p in enumerate(probs):
        paths.append(os.path.join(d, f"p{k}.bin"))
        _write(paths[-1], p)
    # invalid descriptors: a lower-triangle entry, a constraint index past m,
    # a NaN value, coded-diffraction sizes that do not match
    q = si.random_hslr(30, 10, 3)
    q.row, q.col = q.col.copy(), q.row.copy()
    bad = [q]
    q = si.random_hslr(30, 10, 3)
    q.con = q.con.copy()
    q.con[0] = 99
    bad.append(q)
    q = si.random_hslr(30, 10, 3)
    q.val = q.val.copy()
    q.val[1] = np.nan
    bad.append(q)
    for k, p in enumerate(bad):
        paths.append(os.path.join(d, f"b{k}.bin"))
        _write(paths[-1], p)
    cdp = si.phase_retrieval_cdp(16, 3, seed=1)
    paths.append(os.path.join(d, "b_cdp.bin"))
    _write(paths[-1], cdp, m=cdp.m - 1)
    r = subprocess.run([exe] + paths, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.strip().splitlines()
    assert lines[0].startswith("eig ")
    rows = [list(map(int, l.split())) for l in lines[1:]]
    assert len(rows) == len(paths)
    for p, row in zip(probs, rows):
        assert row[0] == 0, row
        s = H.hallar_inspect(p)
        assert (row[1], row[2], row[4], row[5]) == (s["pairs"], s["lower"], s["direct"], s["tiles"]), (row, s)
    assert [row[0] for row in rows[len(probs):]] == [1, 1, 9, 1]
