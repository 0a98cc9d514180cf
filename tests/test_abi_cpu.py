"""C ABI checks that need no GPU: the library loads, exports every function
include/hallar.h declares, validates problem descriptors before touching
the device, and its default solver constants equal the oracle's readings."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import sdp_instances as si
from paper_2505_13719_amd import hallar as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hallar.h")).read()
    return sorted(set(re.findall(r"\b(hallar_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = H.load()
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(H.EXPORTS)


def test_default_options_match_oracle_readings():
    o = H.options()
    ref = oracle.Options()
    for k in ("eps", "beta1", "beta_growth", "beta_max", "infeas_ratio", "pinf_gate", "stall_ratio", "stall_growth", "eps1", "eps_floor",
              "eps_decay", "sigma", "chi", "lam0", "drop_tol", "eig_frac"):
        assert getattr(o, k) == pytest.approx(getattr(ref, k)), k
    # library-only switches: default schedule, lower half recomputed where eligible
    assert o.autotune == 0 and o.lower_gather == 0


def _bad(prob, code):
    with pytest.raises(H.HallarError) as e:
        H.hallar_footprint(prob)
    assert e.value.status == code


def test_descriptor_validation():
    p = si.random_hslr(8, 4, 0)
    # lower-triangle entry
    q = si.random_hslr(8, 4, 0)
    q.row, q.col = q.col.copy(), q.row.copy()
    off = q.row != q.col
    if off.any():
        _bad(q, 1)
    # constraint index beyond m
    q = si.random_hslr(8, 4, 0)
    q.con = q.con.copy(); q.con[0] = 99
    _bad(q, 1)
    # NaN value
    q = si.random_hslr(8, 4, 0)
    q.val = q.val.copy(); q.val[3] = np.nan
    _bad(q, 9)
    # two low-rank objective terms, or one of rank 3: unsupported by the library
    q = si.random_hslr(8, 4, 0)
    q.lr_con = [0, 0]; q.lr_K = [q.lr_K[0], q.lr_K[0]]; q.lr_D = [q.lr_D[0], q.lr_D[0]]
    _bad(q, 2)
    q = si.random_hslr(8, 4, 0)
    q.lr_K = [np.ones((8, 3))]; q.lr_D = [np.eye(3)]
    _bad(q, 2)
    # constraints' low-rank parts beyond 4096 columns in all
    q = si.random_hslr(8, 4, 0)
    q.lr_con = [1, 2]; q.lr_K = [np.ones((8, 2048)), np.ones((8, 2049))]; q.lr_D = [np.eye(2048), np.eye(2049)]
    _bad(q, 2)
    # a low-rank term on a constraint out of range
    q = si.random_hslr(8, 4, 0, lowrank_nonobjective=True)
    q.lr_con = [0, 5]
    _bad(q, 1)
    # low-rank terms on constraints are supported: footprint and structure without a device
    q = si.random_hslr(8, 4, 0, lowrank_nonobjective=True)
    assert H.hallar_footprint(q) > H.hallar_footprint(si.random_hslr(8, 4, 0))
    assert H.hallar_inspect(q)["direct"] == 0
    # a valid one has a positive, deterministic footprint
    b1 = H.hallar_footprint(p)
    b2 = H.hallar_footprint(p)
    assert b1 == b2 > 0
    assert H.hallar_footprint(p, H.FP32_MIXED) < b1


def test_footprint_grows_with_size():
    small = si.maxcut_problem(50, *si.er_edges(50, 0.1, np.random.default_rng(0)))
    big = si.maxcut_problem(500, *si.er_edges(500, 0.1, np.random.default_rng(0)))
    assert H.hallar_footprint(big) > H.hallar_footprint(small)


@pytest.mark.parametrize("field,value", [("lower_gather", 2), ("unfused_trial", -1), ("profile", 3),
                                         ("rank_cap", 65), ("eig_kmax", 65), ("sigma", 0.6)])
def test_option_validation(field, value):
    """hallar_create checks the options before touching the device: an out-of-range
    value gives E_INVALID naming the field."""
    o = H.options(**{field: value})
    with pytest.raises(H.HallarError) as e:
        H.hallar_create(si.random_hslr(8, 4, 0), H.FP64, o, stream=0)  # no device is touched
    assert e.value.status == 1
    assert field in str(e.value)


def test_coded_diffraction_validation():
    """Coded-diffraction problems (Section 5.4, real form): the shapes are
    checked and mixtures refused before any device work."""
    p = si.phase_retrieval_cdp(12, 3, seed=1)
    assert H.hallar_footprint(p) > 0
    assert H.hallar_inspect(p)["direct"] == 0
    q = si.phase_retrieval_cdp(12, 3, seed=1)
    q.m, q.b = q.m - 1, q.b[:-1]                      # m != L n_c
    _bad(q, 1)
    q = si.phase_retrieval_cdp(12, 3, seed=1)
    q.n = q.n + 1                                      # odd n
    _bad(q, 1)
    q = si.phase_retrieval_cdp(12, 3, seed=1)
    q.con = q.con.copy(); q.con[0] = 1                 # a sparse constraint entry
    _bad(q, 2)
    q = si.phase_retrieval_cdp(12, 3, seed=1)
    q.lr_con, q.lr_K, q.lr_D = [0], [np.ones((q.n, 1))], [np.eye(1)]
    _bad(q, 2)
    q = si.phase_retrieval_cdp(12, 3, seed=1)
    q.cdp_masks = q.cdp_masks.copy(); q.cdp_masks[1, 2] = np.nan
    _bad(q, 9)
