"""ctypes binding of the C ABI in include/hallar.h.

Argument marshalling only: every operator, eigen solve and solve runs in the
HIP library (libhallar.so, built in-tree for gfx950).  Device buffers are
torch tensors on a ROCm device; streams are torch streams.  The binding
fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhallar.so")

HALLAR_OK = 0
STATUS = {0: "ok", 1: "invalid", 2: "unsupported", 3: "oom", 4: "hip", 5: "not_converged", 6: "iter_limit",
          7: "time_limit", 8: "rank_cap", 9: "numerical", 10: "busy"}
FP64, FP32_MIXED = 0, 1

i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)
f64p = C.POINTER(C.c_double)


class hallar_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("trace_bound", C.c_double), ("nnz", C.c_int64),
                ("row", i32p), ("col", i32p), ("con", i32p), ("val", f64p),
                ("n_lowrank", C.c_int32), ("lr_con", i32p), ("lr_rank", i32p), ("K_off", i64p), ("D_off", i64p),
                ("K", f64p), ("D", f64p), ("b", f64p), ("cdp_patterns", C.c_int32), ("cdp_masks", f64p)]


class hallar_options(C.Structure):
    _fields_ = [("eps", C.c_double), ("beta1", C.c_double), ("beta_growth", C.c_double), ("beta_max", C.c_double),
                ("infeas_ratio", C.c_double), ("pinf_gate", C.c_double), ("stall_ratio", C.c_double),
                ("stall_growth", C.c_double), ("eps1", C.c_double),
                ("eps_floor", C.c_double), ("eps_decay", C.c_double), ("sigma", C.c_double), ("chi", C.c_double),
                ("lam0", C.c_double), ("fista_max_iter", C.c_int32), ("aipp_max_iter", C.c_int32),
                ("hlr_max_iter", C.c_int32), ("outer_max_iter", C.c_int32), ("eig_tol", C.c_double),
                ("eig_frac", C.c_double), ("eig_kmax", C.c_int32), ("eig_max_iter", C.c_int32),
                ("rank_cap", C.c_int32), ("drop_tol", C.c_double), ("time_limit", C.c_double),
                ("seed", C.c_uint64), ("verbose", C.c_int32), ("profile", C.c_int32), ("autotune", C.c_int32),
                ("lower_gather", C.c_int32), ("unfused_trial", C.c_int32), ("obj_check", C.c_int32),
                ("rank_cap_truncate", C.c_int32), ("graphs", C.c_int32), ("pad_", C.c_int32)]


class hallar_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("rank", C.c_int32), ("outer_iters", C.c_int32), ("pad_", C.c_int32),
                ("pval", C.c_double), ("dval", C.c_double), ("theta", C.c_double), ("pinf", C.c_double),
                ("gap", C.c_double), ("dinf", C.c_double), ("beta", C.c_double), ("seconds", C.c_double),
                ("n_sddmm", C.c_int64), ("n_spmm", C.c_int64), ("n_matvec", C.c_int64),
                ("n_fista_trials", C.c_int64), ("n_aipp_iters", C.c_int64), ("n_hlr_iters", C.c_int64),
                ("n_eig_calls", C.c_int64), ("n_truncations", C.c_int64), ("n_rounds", C.c_int64),
                ("obj_bound", C.c_double), ("n_graph_rounds", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}
        d["status"] = STATUS.get(self.status, str(self.status))
        return d


class hallar_outer_record(C.Structure):
    _fields_ = [("t", C.c_int32), ("rank", C.c_int32), ("beta", C.c_double), ("pval", C.c_double),
                ("dval", C.c_double), ("theta", C.c_double), ("pinf", C.c_double), ("gap", C.c_double),
                ("dinf", C.c_double), ("obj_bound", C.c_double), ("seconds", C.c_double),
                ("n_fista_trials", C.c_int64), ("n_matvec", C.c_int64), ("n_hlr_iters", C.c_int64)]


class hallar_eig_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("residual", C.c_double)]


EXPORTS = ["hallar_default_options", "hallar_create", "hallar_destroy", "hallar_last_error", "hallar_describe",
           "hallar_eval_AUUt", "hallar_eval_AUUt_noalloc", "hallar_adjoint_spmm", "hallar_min_eig", "hallar_solve", "hallar_get_solution",
           "hallar_get_history",
           "hallar_solve_batch", "hallar_footprint", "hallar_pool_create", "hallar_pool_destroy",
           "hallar_pool_admit", "hallar_pool_step", "hallar_pool_poll", "hallar_pool_usage", "hallar_profile",
           "hallar_pool_profile", "hallar_schedule", "hallar_inspect"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libhallar.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python paper_2505_13719_amd/build.py`")
    L = C.CDLL(path)
    vp = C.c_void_p
    L.hallar_default_options.argtypes = [C.POINTER(hallar_options)]
    L.hallar_default_options.restype = None
    L.hallar_create.argtypes = [C.POINTER(hallar_problem), C.c_int, C.POINTER(hallar_options), vp, C.POINTER(vp)]
    L.hallar_destroy.argtypes = [vp]
    L.hallar_last_error.argtypes = [vp]
    L.hallar_last_error.restype = C.c_char_p
    L.hallar_describe.argtypes = [vp, i64p, i64p, i64p]
    L.hallar_schedule.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), i64p]
    L.hallar_eval_AUUt.argtypes = [vp, vp, C.c_int32, C.c_int64, vp, vp]
    L.hallar_eval_AUUt_noalloc.argtypes = [vp, vp, C.c_int32, C.c_int64, vp, vp]
    L.hallar_adjoint_spmm.argtypes = [vp, vp, vp, C.c_int32, C.c_int64, vp, C.c_int64, vp]
    L.hallar_min_eig.argtypes = [vp, vp, vp, C.c_double, C.c_int32, f64p, vp, C.POINTER(hallar_eig_info), vp]
    L.hallar_solve.argtypes = [vp, vp, C.c_int32, vp, C.POINTER(hallar_result)]
    L.hallar_get_solution.argtypes = [vp, vp, C.c_int64, vp, vp]
    L.hallar_get_history.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int32)]
    L.hallar_solve_batch.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp), C.POINTER(hallar_result)]
    L.hallar_footprint.argtypes = [C.POINTER(hallar_problem), C.c_int, C.POINTER(hallar_options), C.POINTER(C.c_size_t)]
    L.hallar_inspect.argtypes = [C.POINTER(hallar_problem), C.POINTER(hallar_structure), i64p, C.c_int64]
    L.hallar_pool_create.argtypes = [C.c_size_t, C.c_int32, C.c_int, C.POINTER(hallar_options), vp, C.POINTER(vp)]
    L.hallar_pool_destroy.argtypes = [vp]
    L.hallar_pool_admit.argtypes = [vp, C.POINTER(hallar_problem), vp, C.c_int64]
    L.hallar_pool_step.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    L.hallar_pool_poll.argtypes = [vp, i64p, C.POINTER(hallar_result), C.c_int32, C.POINTER(C.c_int32)]
    L.hallar_pool_usage.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.hallar_profile.argtypes = [vp, f64p, i64p, f64p, C.c_int32, C.c_int32]
    L.hallar_pool_profile.argtypes = [vp, f64p, i64p, f64p, C.c_int32, C.c_int32]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("hallar_default_options", "hallar_last_error"):
            f.restype = C.c_int
    _lib = L
    return L


class HallarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st, h=None):
    if st != HALLAR_OK:
        msg = load().hallar_last_error(h)
        raise HallarError(st, msg.decode() if msg else "")
    return st


def options(**kw) -> hallar_options:
    o = hallar_options()
    load().hallar_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class _ProblemArrays:
    """Keeps the numpy arrays a hallar_problem points to alive."""

    def __init__(self, prob):
        self.row = np.ascontiguousarray(prob.row, dtype=np.int32)
        self.col = np.ascontiguousarray(prob.col, dtype=np.int32)
        self.con = np.ascontiguousarray(prob.con, dtype=np.int32)
        self.val = np.ascontiguousarray(prob.val, dtype=np.float64)
        self.b = np.ascontiguousarray(prob.b, dtype=np.float64)
        nl = len(prob.lr_con)
        self.lr_con = np.asarray(prob.lr_con, dtype=np.int32)
        self.lr_rank = np.asarray([K.shape[1] for K in prob.lr_K], dtype=np.int32)
        Ks = [np.ascontiguousarray(K, dtype=np.float64).reshape(-1) for K in prob.lr_K]
        Ds = [np.ascontiguousarray(D, dtype=np.float64).reshape(-1) for D in prob.lr_D]
        self.K = np.concatenate(Ks) if Ks else np.zeros(1)
        self.D = np.concatenate(Ds) if Ds else np.zeros(1)
        self.K_off = np.cumsum([0] + [k.size for k in Ks])[:nl].astype(np.int64) if nl else np.zeros(1, np.int64)
        self.D_off = np.cumsum([0] + [d.size for d in Ds])[:nl].astype(np.int64) if nl else np.zeros(1, np.int64)
        p = hallar_problem()
        p.n, p.m, p.trace_bound, p.nnz = int(prob.n), int(prob.m), float(prob.tau2), int(self.row.size)
        p.row = self.row.ctypes.data_as(i32p)
        p.col = self.col.ctypes.data_as(i32p)
        p.con = self.con.ctypes.data_as(i32p)
        p.val = self.val.ctypes.data_as(f64p)
        p.b = self.b.ctypes.data_as(f64p)
        p.n_lowrank = nl
        if nl:
            p.lr_con = self.lr_con.ctypes.data_as(i32p)
            p.lr_rank = self.lr_rank.ctypes.data_as(i32p)
            p.K_off = self.K_off.ctypes.data_as(i64p)
            p.D_off = self.D_off.ctypes.data_as(i64p)
            p.K = self.K.ctypes.data_as(f64p)
            p.D = self.D.ctypes.data_as(f64p)
        masks = getattr(prob, "cdp_masks", None)
        if masks is not None:
            # complex masks as interleaved (re, im) doubles
            self.cdp = np.ascontiguousarray(masks, dtype=np.complex128).view(np.float64).reshape(-1)
            p.cdp_patterns = int(masks.shape[0])
            p.cdp_masks = self.cdp.ctypes.data_as(f64p)
        self.c = p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, name, dtype=None, numel=None, rows=None, cols=None):
    """Validate a device tensor before its pointer crosses the ABI (the C
    side cannot see allocation sizes)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements")
    if rows is not None:
        if t.dim() != 2 or t.shape[0] != rows or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
            raise ValueError(f"{name} must be a row-major ({rows} x r) matrix")
        if cols is not None and t.shape[1] != cols:
            raise ValueError(f"{name} must have {cols} columns")


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ------------------------------------------------------------------ C names
class Handle(C.c_void_p):
    """Handle returned by hallar_create; remembers n, m and the operator type."""


def _optype(h):
    import torch
    return torch.float64 if h.precision == FP64 else torch.float32


def hallar_create(prob, precision=FP64, opts=None, stream=None):
    L = load()
    pa = _ProblemArrays(prob)
    h = Handle()
    st = L.hallar_create(C.byref(pa.c), int(precision), C.byref(opts) if opts is not None else None,
                         _stream(stream), C.byref(h))
    _check(st)
    h.n, h.m, h.precision = int(prob.n), int(prob.m), int(precision)
    return h


def hallar_destroy(h):
    return _check(load().hallar_destroy(h))


def hallar_describe(h):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().hallar_describe(h, C.byref(a), C.byref(b), C.byref(c)), h)
    return dict(pairs=a.value, sym_nnz=b.value, device_bytes=c.value)


def hallar_eval_AUUt(h, U, T, stream=None):
    """T (float64, m+1) <- A~(U U^T); U: n x r row-major (leading dim = U.stride(0))."""
    import torch
    _need(U, "U", _optype(h), rows=h.n)
    _need(T, "T", torch.float64, numel=h.m + 1)
    r = U.shape[1]
    return _check(load().hallar_eval_AUUt(h, _ptr(U), r, U.stride(0), _ptr(T), _stream(stream)), h)


def hallar_eval_AUUt_noalloc(h, U, T, stream=None):
    """As hallar_eval_AUUt, with the library's static per-GPU scratch array
    instead of the handle's workspace (no allocation at call time)."""
    import torch
    _need(U, "U", _optype(h), rows=h.n)
    _need(T, "T", torch.float64, numel=h.m + 1)
    return _check(load().hallar_eval_AUUt_noalloc(h, _ptr(U), U.shape[1], U.stride(0), _ptr(T), _stream(stream)), h)


def hallar_adjoint_spmm(h, p, U, W, stream=None):
    """W <- (C + A*(p)) U."""
    import torch
    _need(U, "U", _optype(h), rows=h.n)
    _need(W, "W", _optype(h), rows=h.n, cols=U.shape[1])
    if h.m > 0:
        _need(p, "p", torch.float64, numel=h.m)
    return _check(load().hallar_adjoint_spmm(h, _ptr(p), _ptr(U), U.shape[1], U.stride(0), _ptr(W), W.stride(0),
                                             _stream(stream)), h)


def hallar_min_eig(h, p, v, v0=None, tol=1e-10, max_iter=20000, stream=None):
    import torch
    if h.m > 0:
        _need(p, "p", torch.float64, numel=h.m)
    if v is not None:
        _need(v, "v", torch.float64, numel=h.n)
    if v0 is not None:
        _need(v0, "v0", torch.float64, numel=h.n)
    lam = C.c_double()
    info = hallar_eig_info()
    st = load().hallar_min_eig(h, _ptr(p), _ptr(v0), tol, max_iter, C.byref(lam), _ptr(v), C.byref(info),
                               _stream(stream))
    if st not in (0, 5):
        _check(st, h)
    return lam.value, dict(iters=info.iters, restarts=info.restarts, residual=info.residual,
                           converged=st == 0)


def hallar_solve(h, U0=None, p0=None):
    import torch
    res = hallar_result()
    r0 = 0
    if U0 is not None:
        U0 = U0.reshape(h.n, -1)
        _need(U0, "U0", torch.float64, rows=h.n)
        if U0.stride(0) != U0.shape[1]:
            raise ValueError("U0 must be contiguous")
        r0 = U0.shape[1]
    if p0 is not None:
        _need(p0, "p0", torch.float64, numel=h.m)
    _check(load().hallar_solve(h, _ptr(U0), r0, _ptr(p0), C.byref(res)), h)
    return res.as_dict()


def hallar_get_solution(h, U=None, p=None, stream=None):
    import torch
    if U is not None:
        _need(U, "U", torch.float64, rows=h.n)
    if p is not None:
        _need(p, "p", torch.float64, numel=h.m)
    ld = 0 if U is None else U.stride(0)
    return _check(load().hallar_get_solution(h, _ptr(U), ld, _ptr(p), _stream(stream)), h)


def hallar_get_history(h):
    """The last solve's outer-iteration records, as a list of dicts."""
    n = C.c_int32(0)
    _check(load().hallar_get_history(h, None, 0, C.byref(n)), h)
    arr = (hallar_outer_record * max(n.value, 1))()
    _check(load().hallar_get_history(h, arr, n.value, C.byref(n)), h)
    return [{k: getattr(arr[i], k) for k, _ in hallar_outer_record._fields_} for i in range(n.value)]


def hallar_solve_batch(handles, U0s=None):
    import torch
    n = len(handles)
    if U0s is not None:
        for h, u in zip(handles, U0s):
            if u is not None:
                _need(u, "U0", torch.float64, numel=h.n)
    arr = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    u0 = None
    if U0s is not None:
        u0 = (C.c_void_p * n)(*[None if u is None else u.data_ptr() for u in U0s])
    res = (hallar_result * n)()
    _check(load().hallar_solve_batch(arr, n, u0, res))
    return [r.as_dict() for r in res]


class hallar_structure(C.Structure):
    _fields_ = [("pairs", C.c_int64), ("lower", C.c_int64), ("tiles", C.c_int64), ("direct", C.c_int32),
                ("con_rule", C.c_int32), ("lower_recompute", C.c_int32), ("pad_", C.c_int32)]


def hallar_inspect(prob):
    """Host-side structure of an instance (no GPU): pair counts, mode flags and
    the default tile schedule's first rows (numpy int64, tiles + 1 entries)."""
    pa = _ProblemArrays(prob)
    out = hallar_structure()
    _check(load().hallar_inspect(C.byref(pa.c), C.byref(out), None, 0))
    rows = np.zeros(out.tiles + 1, dtype=np.int64)
    _check(load().hallar_inspect(C.byref(pa.c), C.byref(out), rows.ctypes.data_as(i64p), rows.size))
    d = {k: getattr(out, k) for k, _ in out._fields_ if k != "pad_"}
    d["tile_row0"] = rows
    return d


def hallar_footprint(prob, precision=FP64, opts=None):
    pa = _ProblemArrays(prob)
    b = C.c_size_t()
    _check(load().hallar_footprint(C.byref(pa.c), int(precision), C.byref(opts) if opts is not None else None,
                                   C.byref(b)))
    return b.value


def hallar_pool_create(hbm_budget, max_active, precision=FP32_MIXED, opts=None, stream=None):
    p = C.c_void_p()
    _check(load().hallar_pool_create(int(hbm_budget), int(max_active), int(precision),
                                     C.byref(opts) if opts is not None else None, _stream(stream), C.byref(p)))
    return p


def hallar_pool_destroy(pool):
    return _check(load().hallar_pool_destroy(pool))


def hallar_pool_admit(pool, prob, ticket, U0=None):
    """Returns 'ok', 'oom' (footprint does not fit now) or 'busy' (no slot)."""
    pa = _ProblemArrays(prob)
    u0 = None
    if U0 is not None:
        U0 = np.ascontiguousarray(U0, dtype=np.float64).reshape(-1)
        u0 = U0.ctypes.data_as(C.c_void_p)
    st = load().hallar_pool_admit(pool, C.byref(pa.c), u0, int(ticket))
    if st in (3, 10):
        return STATUS[st]
    _check(st)
    return "ok"


def hallar_pool_step(pool, rounds=1):
    n = C.c_int32()
    _check(load().hallar_pool_step(pool, int(rounds), C.byref(n)))
    return n.value


def hallar_pool_poll(pool, cap=4096):
    t = (C.c_int64 * cap)()
    r = (hallar_result * cap)()
    nd = C.c_int32()
    _check(load().hallar_pool_poll(pool, t, r, cap, C.byref(nd)))
    return [(t[k], r[k].as_dict()) for k in range(nd.value)]


def hallar_pool_usage(pool):
    u, b = C.c_size_t(), C.c_size_t()
    _check(load().hallar_pool_usage(pool, C.byref(u), C.byref(b)))
    return u.value, b.value


KERNEL_CLASSES = ["sddmm", "spmm", "lanczos_spmv", "lanczos_reorth", "vector", "reduce", "other", "sddmm_spmm",
                  "cdp"]


def _profile(fn, obj, reset):
    n = len(KERNEL_CLASSES)
    ms, nl, by = (C.c_double * n)(), (C.c_int64 * n)(), (C.c_double * n)()
    _check(fn(obj, ms, nl, by, n, 1 if reset else 0))
    return {k: dict(ms=ms[i], launches=nl[i], bytes=by[i]) for i, k in enumerate(KERNEL_CLASSES)}


def hallar_schedule(h):
    """(min_rows, ent_cap, ntiles) of the handle's tile schedule."""
    a, b, c = C.c_int32(), C.c_int32(), C.c_int64()
    _check(load().hallar_schedule(h, C.byref(a), C.byref(b), C.byref(c)), h)
    return a.value, b.value, c.value


def hallar_profile(h, reset=False):
    """Per kernel class: total ms, launches, algorithmic bytes (opts.profile = 1)."""
    return _profile(load().hallar_profile, h, reset)


def hallar_pool_profile(pool, reset=False):
    return _profile(load().hallar_pool_profile, pool, reset)
