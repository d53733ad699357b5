"""ctypes binding of libpsa (include/psa.h).

Argument marshalling only: every computation runs in libpsa's HIP kernels
(or, for the once-per-run schedule and variability draw, in its native host
code).  The raw functions keep the C names (psa_ctx_create, ...); the small
classes below wrap them for numpy / torch callers.  torch is used only for
device memory and streams: a device output is a cuda tensor whose data_ptr()
is handed to the library on the context's stream.

If libpsa.so has not been built this module raises at import time; there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpsa.so")

PSA_OK = 0
PSA_EINVAL = -1
PSA_ENOMEM = -2
PSA_EHIP = -3
PSA_EUNSUPPORTED = -4
PSA_EAGAIN = -5
PSA_ECANCELED = -6
PSA_ETIMEDOUT = -7
PSA_EINTERNAL = -8
PSA_JOB_QUEUED, PSA_JOB_RUNNING, PSA_JOB_DONE, PSA_JOB_ERROR, PSA_JOB_CANCELED = range(5)

PSA_GRAPH_ISING = 0
PSA_GRAPH_MAXCUT = 1
PSA_OUT_HOST = 0
PSA_OUT_DEVICE = 1
PSA_BATCH_SEQUENTIAL = 2
PSA_PATH_AUTO, PSA_PATH_CSR, PSA_PATH_DENSE = 0, 1, 2
PSA_TUNE = 4
PSA_NOALLOC_SCRATCH_BYTES = 128 << 20
PSA_ALG_PSA, PSA_ALG_SPSA, PSA_ALG_TAPSA = 0, 1, 2
PSA_TUNE_ALONE, PSA_TUNE_BATCH = 0, 1
PSA_DENSE_LAUNCH_STEPS, PSA_DENSE_LAUNCH_GRAPH, PSA_DENSE_LAUNCH_PERSISTENT = 0, 1, 2

_P = ctypes.c_void_p
_i32, _i64, _u32, _u64, _f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_double)


class psa_graph_info(ctypes.Structure):
    _fields_ = [("n", _i32), ("edges", _i64), ("nnz", _i64), ("w_total", _i64),
                ("max_abs_field", _i32), ("max_degree", _i32),
                ("unit_weights", _i32), ("mean_s", _f64), ("device_bytes", _i64)]


class psa_run_desc(ctypes.Structure):
    _fields_ = [("steps", _i32), ("trials", _i32), ("seed", _u64),
                ("i0_min", _f64), ("i0_max", _f64), ("i0", _P),
                ("sigma_lambda", _f64), ("sigma_delta", _f64),
                ("sigma_nu", _f64), ("p_mean", _f64), ("lambda_", _P),
                ("delta", _P), ("thr24", _P), ("block", _i32),
                ("trials_per_group", _i32), ("lanes_per_task", _i32), ("flags", _u32),
                ("algorithm", _u32), ("p_stall", _f64), ("window", _i32), ("t_res", _i32),
                ("period", _P)]


class psa_tune_result(ctypes.Structure):
    _fields_ = [("path", _u32), ("trials_per_group", _i32), ("lanes_per_task", _i32),
                ("candidates", _i32), ("us_per_step", _f64), ("csr_us_per_step", _f64),
                ("dense_us_per_step", _f64), ("model_csr_us", _f64), ("model_dense_us", _f64)]


class psa_job_info(ctypes.Structure):
    _fields_ = [("path", _u32), ("trials_per_group", _i32), ("lanes_per_task", _i32),
                ("block", _i32), ("dense_encoding", _i32), ("algorithm", _u32),
                ("device_bytes", _i64), ("period_classes", _i32),
                ("period_resident", _i32)]


class psa_timing(ctypes.Structure):
    _fields_ = [("anneal_ms", _f64), ("batch_ms", _f64), ("dense_ms", _f64),
                ("anneal_launches", _i64), ("batch_launches", _i64), ("dense_launches", _i64),
                ("dense_graph_launches", _i64)]


class psa_batch_item(ctypes.Structure):
    _fields_ = [("graph", _P), ("desc", psa_run_desc), ("energy_out", _P),
                ("cut_out", _P), ("spins_out", _P)]


class psa_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _i64), ("max_resident", _i32), ("quantum_steps", _i32),
                ("max_waiting", _i32)]


class psa_result(ctypes.Structure):
    _fields_ = [("status", _i32), ("error", _i32), ("submit_us", _i64), ("admit_us", _i64),
                ("start_us", _i64), ("end_us", _i64)]


class psa_server_stats(ctypes.Structure):
    _fields_ = [("waiting", _i32), ("resident", _i32), ("completed", _i64), ("failed", _i64),
                ("canceled", _i64), ("quanta", _i64), ("used_bytes", _i64),
                ("budget_bytes", _i64), ("peak_resident", _i32), ("peak_used_bytes", _i64)]


# (name, restype, argtypes) of every exported entry point in include/psa.h
_SIGNATURES = [
    ("psa_version", ctypes.c_char_p, []),
    ("psa_last_error", ctypes.c_char_p, []),
    ("psa_ctx_create", _i32, [_i32, _P, ctypes.POINTER(_P)]),
    ("psa_ctx_synchronize", _i32, [_P]),
    ("psa_ctx_destroy", None, [_P]),
    ("psa_ctx_set_timing", _i32, [_P, _i32]),
    ("psa_ctx_timing_read", _i32, [_P, ctypes.POINTER(psa_timing)]),
    ("psa_ctx_set_dense_launch", _i32, [_P, _i32]),
    ("psa_debug_dense_wait_limit", _i32, [_P, _u32]),
    ("psa_graph_from_edges", _i32, [_P, _i32, _i64, _P, _P, _P, _P, _u32,
                                    ctypes.POINTER(_P)]),
    ("psa_graph_from_csr", _i32, [_P, _i32, _P, _P, _P, _P, _u32,
                                  ctypes.POINTER(_P)]),
    ("psa_graph_info_get", _i32, [_P, ctypes.POINTER(psa_graph_info)]),
    ("psa_graph_check_edges", _i32, [_i32, _i64, _P, _P, _P, _P, _u32,
                                     ctypes.POINTER(psa_graph_info)]),
    ("psa_graph_destroy", None, [_P]),
    ("psa_schedule_paper", _i32, [_P, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
    ("psa_schedule_fill", _i32, [_i32, _f64, _f64, _P]),
    ("psa_periods_draw", _i32, [_i32, _u64, _f64, _i32, _P]),
    ("psa_variability_draw", _i32, [_i32, _u64, _f64, _f64, _f64, _f64, _P, _P, _P]),
    ("psa_run_desc_default", None, [ctypes.POINTER(psa_run_desc)]),
    ("psa_job_create", _i32, [_P, _P, ctypes.POINTER(psa_run_desc), ctypes.POINTER(_P)]),
    ("psa_job_reset", _i32, [_P]),
    ("psa_job_step", _i32, [_P, _i32]),
    ("psa_job_position", _i32, [_P, ctypes.POINTER(_i32)]),
    ("psa_job_get_info", _i32, [_P, ctypes.POINTER(psa_job_info)]),
    ("psa_job_read_spins", _i32, [_P, _P, _u32]),
    ("psa_job_write_spins", _i32, [_P, _P, _i32, _u32]),
    ("psa_job_local_field", _i32, [_P, _P, _u32]),
    ("psa_job_energy_cut", _i32, [_P, _P, _P, _u32]),
    ("psa_job_destroy", None, [_P]),
    ("psa_anneal", _i32, [_P, _P, ctypes.POINTER(psa_run_desc), _P, _P, _P, _u32]),
    ("psa_anneal_noalloc", _i32, [_P, _P, ctypes.POINTER(psa_run_desc), _P, _P, _P]),
    ("psa_jobs_step_batch", _i32, [_P, _i32, ctypes.POINTER(_P), _i32]),
    ("psa_jobs_energy_cut", _i32, [_P, _i32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                   ctypes.POINTER(_P), _u32]),
    ("psa_anneal_batch", _i32, [_P, _i32, ctypes.POINTER(psa_batch_item), _u32]),
    ("psa_autotune", _i32, [_P, _P, ctypes.POINTER(psa_run_desc), _i32, _u32,
                            ctypes.POINTER(psa_tune_result)]),
    ("psa_tune_get", _i32, [_P, _P, ctypes.POINTER(psa_run_desc), _u32,
                            ctypes.POINTER(psa_tune_result)]),
    ("psa_tune_apply", None, [ctypes.POINTER(psa_tune_result), ctypes.POINTER(psa_run_desc)]),
    ("psa_tune_cache_size", _i32, [_P]),
    ("psa_tune_clear", None, [_P]),
    ("psa_server_create", _i32, [_P, ctypes.POINTER(psa_server_opts), ctypes.POINTER(_P)]),
    ("psa_server_submit", _i32, [_P, _i32, _i64, _P, _P, _P, _P, _u32,
                                 ctypes.POINTER(psa_run_desc), _P, _P, _P,
                                 ctypes.POINTER(_u64)]),
    ("psa_server_poll", _i32, [_P, _u64, ctypes.POINTER(psa_result)]),
    ("psa_server_wait", _i32, [_P, _u64, _i64, ctypes.POINTER(psa_result)]),
    ("psa_server_cancel", _i32, [_P, _u64]),
    ("psa_server_release", _i32, [_P, _u64]),
    ("psa_server_stats_get", _i32, [_P, ctypes.POINTER(psa_server_stats)]),
    ("psa_server_destroy", None, [_P]),
    ("psa_debug_tanh", _i32, [_P, _i64, _P, _P]),
    ("psa_debug_decide", _i32, [_P, _i64, _P, _P, _P]),
]


def _load():
    # torch bundles its own HIP runtime (same SONAME as ROCm's).  Loading it
    # first makes libpsa bind to that one copy, so device pointers and
    # streams can be shared with torch; otherwise the process would end up
    # with two HIP runtimes and torch would not see the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`"
            " (the pSA path has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in _SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = [s[0] for s in _SIGNATURES]


class PsaError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where} failed ({status}): {message}")
        self.status = status


def _check(status, where):
    if status != PSA_OK:
        raise PsaError(status, where, _lib.psa_last_error().decode(errors="replace"))


# ----------------------------------------------------------------------------
# Raw entry points under their C names (thin pass-through).
# ----------------------------------------------------------------------------
def __getattr__(name):
    if name in EXPORTED:
        return getattr(_lib, name)
    raise AttributeError(name)


def _ptr(a):
    """Address of a numpy array, a torch tensor, or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data_as(_P)
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return _P(a.data_ptr())
    raise TypeError(f"unsupported buffer type {type(a)!r}")


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _flags_for(*bufs):
    dev = [_is_device(b) for b in bufs if b is not None]
    if dev and any(dev) != all(dev):
        raise ValueError("outputs must all be host or all be device buffers")
    return PSA_OUT_DEVICE if dev and dev[0] else PSA_OUT_HOST


def version():
    return _lib.psa_version().decode()


class Context:
    """HIP device + stream.  `stream` may be a torch.cuda.Stream, a raw
    hipStream_t address, or None (the library creates one)."""

    def __init__(self, device=0, stream=None):
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = _P()
        _check(_lib.psa_ctx_create(device, _P(stream) if stream else None,
                                   ctypes.byref(h)), "psa_ctx_create")
        self.handle = h
        self.device = device

    def set_timing(self, on=True):
        """Record device time per kernel family (psa_ctx_set_timing)."""
        _check(_lib.psa_ctx_set_timing(self.handle, 1 if on else 0), "psa_ctx_set_timing")

    def set_dense_launch(self, how):
        """How dense quanta are launched (psa_ctx_set_dense_launch): one of
        PSA_DENSE_LAUNCH_STEPS, _GRAPH, _PERSISTENT."""
        _check(_lib.psa_ctx_set_dense_launch(self.handle, int(how)), "psa_ctx_set_dense_launch")

    def debug_dense_wait_limit(self, max_polls):
        """Bound of the persistent dense launch's dependency waits (psa_debug_dense_wait_limit)."""
        _check(_lib.psa_debug_dense_wait_limit(self.handle, int(max_polls)), "psa_debug_dense_wait_limit")

    def timing(self):
        """Totals since the last call (psa_ctx_timing_read), as a dict."""
        r = psa_timing()
        _check(_lib.psa_ctx_timing_read(self.handle, ctypes.byref(r)), "psa_ctx_timing_read")
        return {f: getattr(r, f) for f, _ in psa_timing._fields_}

    def synchronize(self):
        _check(_lib.psa_ctx_synchronize(self.handle), "psa_ctx_synchronize")

    def close(self):
        if self.handle:
            _lib.psa_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle

    @classmethod
    def from_edges(cls, ctx, n, u, v, val, h=None, maxcut=True):
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.int32)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
        if not (u.shape == v.shape == val.shape) or (hh is not None and hh.shape != (n,)):
            raise ValueError("edge arrays must have equal length and h shape (n,)")
        out = _P()
        _check(_lib.psa_graph_from_edges(ctx.handle, n, u.size, _ptr(u), _ptr(v),
                                         _ptr(val), _ptr(hh),
                                         PSA_GRAPH_MAXCUT if maxcut else PSA_GRAPH_ISING,
                                         ctypes.byref(out)), "psa_graph_from_edges")
        return cls(ctx, out)

    @classmethod
    def from_csr(cls, ctx, n, row_ptr, col, val, h=None, maxcut=False):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.int32)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
        out = _P()
        _check(_lib.psa_graph_from_csr(ctx.handle, n, _ptr(rp), _ptr(col), _ptr(val),
                                       _ptr(hh),
                                       PSA_GRAPH_MAXCUT if maxcut else PSA_GRAPH_ISING,
                                       ctypes.byref(out)), "psa_graph_from_csr")
        return cls(ctx, out)

    def info(self):
        i = psa_graph_info()
        _check(_lib.psa_graph_info_get(self.handle, ctypes.byref(i)), "psa_graph_info_get")
        return {f: getattr(i, f) for f, _ in psa_graph_info._fields_}

    def schedule_paper(self):
        lo, hi = _f64(), _f64()
        _check(_lib.psa_schedule_paper(self.handle, ctypes.byref(lo), ctypes.byref(hi)),
               "psa_schedule_paper")
        return lo.value, hi.value

    def close(self):
        if self.handle:
            _lib.psa_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_check_edges(n, u, v, val, h=None, maxcut=True):
    """Validate an edge list on the host and return its statistics
    (psa_graph_check_edges; no context or device needed)."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.int32)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
    if not (u.shape == v.shape == val.shape) or (hh is not None and hh.shape != (n,)):
        raise ValueError("edge arrays must have equal length and h shape (n,)")
    i = psa_graph_info()
    _check(_lib.psa_graph_check_edges(n, u.size, _ptr(u), _ptr(v), _ptr(val), _ptr(hh),
                                      PSA_GRAPH_MAXCUT if maxcut else PSA_GRAPH_ISING,
                                      ctypes.byref(i)), "psa_graph_check_edges")
    return {f: getattr(i, f) for f, _ in psa_graph_info._fields_}


def schedule_fill(steps, i0_min, i0_max):
    out = np.zeros(max(int(steps), 1), np.float32)
    _check(_lib.psa_schedule_fill(int(steps), float(i0_min), float(i0_max), _ptr(out)),
           "psa_schedule_fill")
    return out[:steps]


def periods_draw(n, seed, sigma_nu, t_res):
    """Integer timing periods of the period mode (psa_periods_draw)."""
    out = np.zeros(n, np.uint32)
    _check(_lib.psa_periods_draw(int(n), int(seed), float(sigma_nu), int(t_res), _ptr(out)),
           "psa_periods_draw")
    return out


def variability_draw(n, seed, sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0, p_mean=1.0):
    lam = np.zeros(n, np.float32)
    dlt = np.zeros(n, np.float32)
    thr = np.zeros(n, np.uint32)
    _check(_lib.psa_variability_draw(n, seed, sigma_lambda, sigma_delta, sigma_nu, p_mean,
                                     _ptr(lam), _ptr(dlt), _ptr(thr)), "psa_variability_draw")
    return lam, dlt, thr


def make_desc(steps, trials, seed=0, i0=None, i0_min=None, i0_max=None,
              sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0, p_mean=1.0,
              lam=None, delta=None, thr24=None, block=0, trials_per_group=0,
              lanes_per_task=0, path=PSA_PATH_AUTO, tune=False, algorithm=PSA_ALG_PSA,
              p_stall=0.5, window=4, t_res=0, period=None):
    """Build a psa_run_desc; returns (desc, keepalive arrays).  tune=True sets
    PSA_TUNE (path and launch shape from the context's tuning cache)."""
    d = psa_run_desc()
    _lib.psa_run_desc_default(ctypes.byref(d))
    d.steps, d.trials, d.seed = int(steps), int(trials), int(seed)
    keep = []
    if i0 is not None:
        a = np.ascontiguousarray(i0, dtype=np.float32)
        keep.append(a)
        d.i0 = _ptr(a)
    if i0_min is not None:
        d.i0_min, d.i0_max = float(i0_min), float(i0_max)
    d.sigma_lambda, d.sigma_delta, d.sigma_nu = float(sigma_lambda), float(sigma_delta), float(sigma_nu)
    d.p_mean = float(p_mean)
    for field, arr, dt in (("lambda_", lam, np.float32), ("delta", delta, np.float32),
                           ("thr24", thr24, np.uint32)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=dt)
            keep.append(a)
            setattr(d, field, _ptr(a))
    d.block = int(block)
    d.trials_per_group = int(trials_per_group)
    d.lanes_per_task = int(lanes_per_task)
    d.flags = int(path) | (PSA_TUNE if tune else 0)
    d.algorithm = int(algorithm)
    d.p_stall = float(p_stall)
    d.window = int(window)
    d.t_res = int(t_res)
    if period is not None:
        a = np.ascontiguousarray(period, dtype=np.uint32)
        keep.append(a)
        d.period = _ptr(a)
    return d, keep


def autotune(ctx, graph, steps, trials, seed=0, probe_steps=8, batch=False, **kw):
    """Time the applicable paths and launch shapes (psa_autotune); returns a
    dict of the psa_tune_result fields."""
    desc, keep = make_desc(steps, trials, seed, **kw)
    r = psa_tune_result()
    _check(_lib.psa_autotune(ctx.handle, graph.handle, ctypes.byref(desc), int(probe_steps),
                             PSA_TUNE_BATCH if batch else PSA_TUNE_ALONE, ctypes.byref(r)),
           "psa_autotune")
    del keep
    return {f: getattr(r, f) for f, _ in psa_tune_result._fields_}


def tune_get(ctx, graph, steps, trials, seed=0, batch=False, **kw):
    """The tuning cache's entry for this graph's shape class (measured on a
    miss, psa_tune_get); returns a dict of the psa_tune_result fields."""
    desc, keep = make_desc(steps, trials, seed, **kw)
    r = psa_tune_result()
    _check(_lib.psa_tune_get(ctx.handle, graph.handle, ctypes.byref(desc),
                             PSA_TUNE_BATCH if batch else PSA_TUNE_ALONE, ctypes.byref(r)),
           "psa_tune_get")
    del keep
    return {f: getattr(r, f) for f, _ in psa_tune_result._fields_}


def tune_kwargs(r):
    """make_desc keyword arguments that apply a tuning result."""
    return dict(path=r["path"], trials_per_group=r["trials_per_group"],
                lanes_per_task=r["lanes_per_task"])


def tune_cache_size(ctx):
    return int(_lib.psa_tune_cache_size(ctx.handle))


def tune_clear(ctx):
    _lib.psa_tune_clear(ctx.handle)


class Job:
    def __init__(self, ctx, graph, steps, trials, seed=0, **kw):
        self.ctx, self.graph = ctx, graph
        self.n = graph.info()["n"]
        self.trials, self.steps = int(trials), int(steps)
        desc, keep = make_desc(steps, trials, seed, **kw)
        out = _P()
        _check(_lib.psa_job_create(ctx.handle, graph.handle, ctypes.byref(desc),
                                   ctypes.byref(out)), "psa_job_create")
        del keep
        self.handle = out

    def info(self):
        r = psa_job_info()
        _check(_lib.psa_job_get_info(self.handle, ctypes.byref(r)), "psa_job_get_info")
        return {f: getattr(r, f) for f, _ in psa_job_info._fields_}

    @property
    def dense(self):
        return self.info()["path"] == PSA_PATH_DENSE

    def reset(self):
        _check(_lib.psa_job_reset(self.handle), "psa_job_reset")

    def step(self, k):
        _check(_lib.psa_job_step(self.handle, int(k)), "psa_job_step")

    @property
    def position(self):
        t = _i32()
        _check(_lib.psa_job_position(self.handle, ctypes.byref(t)), "psa_job_position")
        return t.value

    def read_spins(self, out=None):
        if out is None:
            out = np.zeros((self.trials, self.n), np.int8)
        _check(_lib.psa_job_read_spins(self.handle, _ptr(out), _flags_for(out)),
               "psa_job_read_spins")
        return out

    def write_spins(self, spins, t):
        if not _is_device(spins):
            spins = np.ascontiguousarray(spins, dtype=np.int8)
        _check(_lib.psa_job_write_spins(self.handle, _ptr(spins), int(t), _flags_for(spins)),
               "psa_job_write_spins")

    def local_field(self, out=None):
        if out is None:
            out = np.zeros((self.trials, self.n), np.int32)
        _check(_lib.psa_job_local_field(self.handle, _ptr(out), _flags_for(out)),
               "psa_job_local_field")
        return out

    def energy_cut(self, energy=None, cut=None):
        if energy is None:
            energy = np.zeros(self.trials, np.int64)
            cut = np.zeros(self.trials, np.int64)
        _check(_lib.psa_job_energy_cut(self.handle, _ptr(energy), _ptr(cut),
                                       _flags_for(energy, cut)), "psa_job_energy_cut")
        return energy, cut

    def close(self):
        if self.handle:
            _lib.psa_job_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def anneal(ctx, graph, steps, trials, seed=0, spins=True, **kw):
    """Whole anneal; returns (spins [trials][n] or None, energy, cut) on the host."""
    n = graph.info()["n"]
    desc, keep = make_desc(steps, trials, seed, **kw)
    E = np.zeros(trials, np.int64)
    C = np.zeros(trials, np.int64)
    S = np.zeros((trials, n), np.int8) if spins else None
    _check(_lib.psa_anneal(ctx.handle, graph.handle, ctypes.byref(desc), _ptr(S), _ptr(E),
                           _ptr(C), PSA_OUT_HOST), "psa_anneal")
    del keep
    return S, E, C


def anneal_noalloc(ctx, graph, steps, trials, seed=0, spins_out=None, energy_out=None,
                   cut_out=None, **kw):
    """Whole anneal with no device allocation (psa_anneal_noalloc): outputs are
    device tensors on the context's device -- energy_out, cut_out int64
    [trials] (required), spins_out int8 [trials][n] or None -- written
    before return."""
    for name, buf in (("energy_out", energy_out), ("cut_out", cut_out), ("spins_out", spins_out)):
        if buf is not None and not _is_device(buf):
            raise ValueError(f"{name} must be a device tensor")
    desc, keep = make_desc(steps, trials, seed, **kw)
    _check(_lib.psa_anneal_noalloc(ctx.handle, graph.handle, ctypes.byref(desc), _ptr(spins_out),
                                   _ptr(energy_out), _ptr(cut_out)), "psa_anneal_noalloc")
    del keep


def jobs_step_batch(ctx, jobs, k):
    """Advance several jobs by up to k steps each in one batched launch."""
    arr = (_P * len(jobs))(*[j.handle for j in jobs])
    _check(_lib.psa_jobs_step_batch(ctx.handle, len(jobs), arr, int(k)), "psa_jobs_step_batch")


def jobs_energy_cut(ctx, jobs, energies=None, cuts=None):
    """Energy and cut of several jobs in one batched read-out.  energies,
    cuts: one int64 [trials] buffer per job (all host numpy or all device
    torch), or None for new host arrays.  Returns (energies, cuts)."""
    if energies is None:
        energies = [np.zeros(j.trials, np.int64) for j in jobs]
        cuts = [np.zeros(j.trials, np.int64) for j in jobs]
    if len(energies) != len(jobs) or len(cuts) != len(jobs):
        raise ValueError("one energy and one cut buffer per job")
    flags = _flags_for(*energies, *cuts) if jobs else PSA_OUT_HOST
    count = len(jobs)
    arr = (_P * count)(*[j.handle for j in jobs])
    ep = (_P * count)(*[_ptr(e) for e in energies])
    cp = (_P * count)(*[_ptr(c) for c in cuts])
    _check(_lib.psa_jobs_energy_cut(ctx.handle, count, arr, ep, cp, flags), "psa_jobs_energy_cut")
    return energies, cuts


def anneal_batch(ctx, items, sequential=False, spins=False):
    """items: list of (graph, steps, trials, seed, kwargs for make_desc).
    Returns a list of (spins or None, energy, cut) host arrays."""
    keep = []
    arr = (psa_batch_item * len(items))()
    outs = []
    for idx, (graph, steps, trials, seed, kw) in enumerate(items):
        desc, k = make_desc(steps, trials, seed, **kw)
        keep.append(k)
        n = graph.info()["n"]
        E = np.zeros(trials, np.int64)
        C = np.zeros(trials, np.int64)
        S = np.zeros((trials, n), np.int8) if spins else None
        outs.append((S, E, C))
        arr[idx].graph = graph.handle
        arr[idx].desc = desc
        arr[idx].energy_out = _ptr(E)
        arr[idx].cut_out = _ptr(C)
        arr[idx].spins_out = _ptr(S)
    flags = PSA_OUT_HOST | (PSA_BATCH_SEQUENTIAL if sequential else 0)
    _check(_lib.psa_anneal_batch(ctx.handle, len(items), arr, flags), "psa_anneal_batch")
    del keep
    return outs


class Server:
    """Continuous-batching anneal server on a context (see psa_server_create)."""

    def __init__(self, ctx, hbm_budget_bytes=0, max_resident=0, quantum_steps=0, max_waiting=0):
        o = psa_server_opts(int(hbm_budget_bytes), int(max_resident), int(quantum_steps),
                            int(max_waiting))
        h = _P()
        _check(_lib.psa_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(h)),
               "psa_server_create")
        self.ctx, self.handle = ctx, h
        self._pending = {}

    def submit(self, n, u, v, val, steps, trials, seed=0, h=None, maxcut=True, spins=False,
               **kw):
        """Queue one anneal; returns a ticket.  The result buffers live in this
        object until result() hands them out."""
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.int32)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
        desc, keep = make_desc(steps, trials, seed, **kw)
        E = np.zeros(trials, np.int64)
        C = np.zeros(trials, np.int64)
        S = np.zeros((trials, n), np.int8) if spins else None
        t = _u64()
        _check(_lib.psa_server_submit(self.handle, n, u.size, _ptr(u), _ptr(v), _ptr(val),
                                      _ptr(hh), PSA_GRAPH_MAXCUT if maxcut else PSA_GRAPH_ISING,
                                      ctypes.byref(desc), _ptr(E), _ptr(C), _ptr(S),
                                      ctypes.byref(t)), "psa_server_submit")
        del keep
        self._pending[t.value] = (S, E, C)
        return t.value

    def poll(self, ticket):
        r = psa_result()
        _check(_lib.psa_server_poll(self.handle, ticket, ctypes.byref(r)), "psa_server_poll")
        return r

    def wait(self, ticket, timeout_s=None):
        """Block until the job ends; returns the psa_result (status field), or
        raises PsaError(PSA_ETIMEDOUT) after timeout_s seconds."""
        r = psa_result()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        _check(_lib.psa_server_wait(self.handle, ticket, us, ctypes.byref(r)), "psa_server_wait")
        return r

    def result(self, ticket):
        """(spins or None, energy, cut) of a finished job; frees its record."""
        r = self.wait(ticket)
        out = self._pending.pop(ticket)
        _check(_lib.psa_server_release(self.handle, ticket), "psa_server_release")
        return r, out

    def cancel(self, ticket):
        _check(_lib.psa_server_cancel(self.handle, ticket), "psa_server_cancel")

    def stats(self):
        st = psa_server_stats()
        _check(_lib.psa_server_stats_get(self.handle, ctypes.byref(st)), "psa_server_stats_get")
        return {f: getattr(st, f) for f, _ in psa_server_stats._fields_}

    def close(self):
        if self.handle:
            _lib.psa_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
