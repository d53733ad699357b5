"""ctypes front end of the pSA oracle (psa_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain single-threaded C
restatement of p-bit simulated annealing with device variability
(Onizawa & Hanyu, arXiv 2601.14476, Methods: Eq. 1-7 and the
SimulatedAnnealingModule listing).  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and this module never imports the GPU library.

Arrays are numpy; the C functions run with the GIL released (ctypes), so
independent trial ranges can be spread over host threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psa_oracle.c")
_LIB = os.path.join(_HERE, "libpsa_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_double)
    lib.psa_ref_philox4x32_10.argtypes = [P, P, P]
    lib.psa_ref_philox4x32_10.restype = None
    lib.psa_ref_word.argtypes = [u64, u32, u32, u32, u32]
    lib.psa_ref_word.restype = u32
    lib.psa_ref_r_from_word.argtypes = [u32]
    lib.psa_ref_r_from_word.restype = ctypes.c_float
    lib.psa_ref_gate.argtypes = [u32, u32]
    lib.psa_ref_gate.restype = ctypes.c_int
    lib.psa_ref_tanh.argtypes = [ctypes.c_float]
    lib.psa_ref_tanh.restype = ctypes.c_float
    lib.psa_ref_tanh_array.argtypes = [i64, P, P]
    lib.psa_ref_tanh_array.restype = None
    lib.psa_ref_r_array.argtypes = [i64, P, P]
    lib.psa_ref_r_array.restype = None
    lib.psa_ref_mean_s.argtypes = [i32, i64, P, P, P, P]
    lib.psa_ref_mean_s.restype = ctypes.c_int
    lib.psa_ref_schedule.argtypes = [i32, f64, f64, P]
    lib.psa_ref_schedule.restype = ctypes.c_int
    lib.psa_ref_variability.argtypes = [i32, u64, f64, f64, f64, f64, P, P, P]
    lib.psa_ref_variability.restype = ctypes.c_int
    lib.psa_ref_init_spins.argtypes = [i32, u64, i32, i32, P]
    lib.psa_ref_init_spins.restype = ctypes.c_int
    lib.psa_ref_local_field.argtypes = [i32, i64, P, P, P, P, i32, P, P]
    lib.psa_ref_local_field.restype = ctypes.c_int
    lib.psa_ref_run.argtypes = [i32, i64, P, P, P, P, P, P, P, P, u64, i32, i32,
                                i32, i32, P]
    lib.psa_ref_run.restype = ctypes.c_int
    lib.psa_ref_run_spsa.argtypes = [i32, i64, P, P, P, P, P, P, P, P, u32, u64, i32,
                                     i32, i32, i32, P, P]
    lib.psa_ref_run_spsa.restype = ctypes.c_int
    lib.psa_ref_run_tapsa.argtypes = [i32, i64, P, P, P, P, P, P, P, P, i32, u64, i32,
                                      i32, i32, i32, P, P]
    lib.psa_ref_run_tapsa.restype = ctypes.c_int
    lib.psa_ref_periods.argtypes = [i32, u64, f64, i32, P]
    lib.psa_ref_periods.restype = ctypes.c_int
    lib.psa_ref_run_period.argtypes = [i32, i64, P, P, P, P, P, P, P, P, i32, u64, i32, i32,
                                       i32, i32, P]
    lib.psa_ref_run_period.restype = ctypes.c_int
    lib.psa_ref_energy_cut.argtypes = [i32, i64, P, P, P, P, i32, P, P, P]
    lib.psa_ref_energy_cut.restype = ctypes.c_int
    lib.psa_ref_anneal.argtypes = [i32, i64, P, P, P, P, i32, P, P, P, P, u64,
                                   i32, i32, P, P, P]
    lib.psa_ref_anneal.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _edges(eu, ev, ej):
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    ej = np.ascontiguousarray(ej, dtype=np.int32)
    if not (eu.shape == ev.shape == ej.shape) or eu.ndim != 1:
        raise ValueError("edge arrays must be 1-D of equal length")
    return eu, ev, ej


def _opt_h(h, n):
    if h is None:
        return None
    h = np.ascontiguousarray(h, dtype=np.int32)
    if h.shape != (n,):
        raise ValueError("h must have shape (n,)")
    return h


TAG_INIT, TAG_R, TAG_GATE, TAG_VAR = 0, 1, 2, 3


def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter and 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.psa_ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def word(seed, t, i, k, tag):
    return int(_load().psa_ref_word(seed, t, i, k, tag))


def r_from_word(u):
    return np.float32(_load().psa_ref_r_from_word(int(u)))


def gate(u, thr24):
    return bool(_load().psa_ref_gate(int(u), int(thr24)))


def tanh(x):
    return np.float32(_load().psa_ref_tanh(float(np.float32(x))))


def tanh_array(xs):
    xs = np.ascontiguousarray(xs, dtype=np.float32)
    out = np.empty_like(xs)
    _load().psa_ref_tanh_array(xs.size, _ptr(xs), _ptr(out))
    return out


def r_array(words):
    words = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.empty(words.shape, np.float32)
    _load().psa_ref_r_array(words.size, _ptr(words), _ptr(out))
    return out


def mean_s(n, eu, ev, ej):
    eu, ev, ej = _edges(eu, ev, ej)
    out = ctypes.c_double()
    _check(_load().psa_ref_mean_s(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej),
                                  ctypes.byref(out)), "psa_ref_mean_s")
    return out.value


def schedule(steps, i0_min, i0_max):
    out = np.zeros(max(steps, 1), np.float32)
    _check(_load().psa_ref_schedule(steps, i0_min, i0_max, _ptr(out)),
           "psa_ref_schedule")
    return out[:steps]


def schedule_paper(n, eu, ev, ej, steps):
    """I0min = 0.1/mean(s), I0max = 10/mean(s) and the geometric schedule."""
    ms = mean_s(n, eu, ev, ej)
    i0_min, i0_max = 0.1 / ms, 10.0 / ms
    return schedule(steps, i0_min, i0_max), i0_min, i0_max


def variability(n, seed, sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0,
                p_mean=1.0):
    lam = np.zeros(n, np.float32)
    off = np.zeros(n, np.float32)
    thr = np.zeros(n, np.uint32)
    _check(_load().psa_ref_variability(n, seed, sigma_lambda, sigma_delta,
                                       sigma_nu, p_mean, _ptr(lam), _ptr(off),
                                       _ptr(thr)), "psa_ref_variability")
    return lam, off, thr


def init_spins(n, seed, trial_begin, trial_end):
    out = np.zeros((trial_end - trial_begin, n), np.int8)
    _check(_load().psa_ref_init_spins(n, seed, trial_begin, trial_end,
                                      _ptr(out)), "psa_ref_init_spins")
    return out


def local_field(n, eu, ev, ej, h, spins):
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    spins = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1, n)
    out = np.zeros(spins.shape, np.int32)
    _check(_load().psa_ref_local_field(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej),
                                       _ptr(h), spins.shape[0], _ptr(spins),
                                       _ptr(out)), "psa_ref_local_field")
    return out


def run(n, eu, ev, ej, h, i0, lam, off, thr, seed, trial_begin, trial_end,
        t_begin, t_end, spins):
    """Sweeps t_begin..t_end-1 on a copy of `spins` ([trials][n])."""
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    i0 = np.ascontiguousarray(i0, dtype=np.float32)
    lam = np.ascontiguousarray(lam, dtype=np.float32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    if i0.size < t_end or lam.size != n or off.size != n or thr.size != n:
        raise ValueError("schedule or per-p-bit arrays have the wrong size")
    s = np.array(spins, dtype=np.int8, copy=True).reshape(trial_end - trial_begin, n)
    s = np.ascontiguousarray(s)
    _check(_load().psa_ref_run(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej), _ptr(h),
                               _ptr(i0), _ptr(lam), _ptr(off), _ptr(thr), seed,
                               trial_begin, trial_end, t_begin, t_end, _ptr(s)),
           "psa_ref_run")
    return s


def run_spsa(n, eu, ev, ej, h, i0, lam, off, thr, stall24, seed, trial_begin, trial_end,
             t_begin, t_end, spins, x_state=None):
    """SpSA sweeps t_begin..t_end-1 (Eq. 5) on copies of `spins` and of the
    held inputs `x_state` ([trials][n] float32; needed when t_begin > 0).
    Returns (spins, x_state)."""
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    i0 = np.ascontiguousarray(i0, dtype=np.float32)
    lam = np.ascontiguousarray(lam, dtype=np.float32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    if i0.size < t_end or lam.size != n or off.size != n or thr.size != n:
        raise ValueError("schedule or per-p-bit arrays have the wrong size")
    rows = trial_end - trial_begin
    s = np.ascontiguousarray(np.array(spins, dtype=np.int8, copy=True).reshape(rows, n))
    if x_state is None:
        if t_begin > 0:
            raise ValueError("x_state is needed to resume at t_begin > 0")
        x = np.zeros((rows, n), np.float32)
    else:
        x = np.ascontiguousarray(np.array(x_state, dtype=np.float32, copy=True).reshape(rows, n))
    _check(_load().psa_ref_run_spsa(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej), _ptr(h),
                                    _ptr(i0), _ptr(lam), _ptr(off), _ptr(thr), int(stall24),
                                    seed, trial_begin, trial_end, t_begin, t_end, _ptr(s),
                                    _ptr(x)),
           "psa_ref_run_spsa")
    return s, x


def periods(n, seed, sigma_nu, t_res):
    """Integer timing periods in sub-steps (psa_ref_periods)."""
    out = np.zeros(n, np.uint32)
    _check(_load().psa_ref_periods(n, seed, float(sigma_nu), int(t_res), _ptr(out)),
           "psa_ref_periods")
    return out


def run_period(n, eu, ev, ej, h, i0, lam, off, period, t_res, seed, trial_begin, trial_end,
               t_begin, t_end, spins):
    """Period-mode cycles t_begin..t_end-1 on a copy of `spins`."""
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    i0 = np.ascontiguousarray(i0, dtype=np.float32)
    lam = np.ascontiguousarray(lam, dtype=np.float32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    period = np.ascontiguousarray(period, dtype=np.uint32)
    if i0.size < t_end or lam.size != n or off.size != n or period.size != n:
        raise ValueError("schedule or per-p-bit arrays have the wrong size")
    rows = trial_end - trial_begin
    s = np.ascontiguousarray(np.array(spins, dtype=np.int8, copy=True).reshape(rows, n))
    _check(_load().psa_ref_run_period(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej), _ptr(h),
                                      _ptr(i0), _ptr(lam), _ptr(off), _ptr(period), int(t_res),
                                      seed, trial_begin, trial_end, t_begin, t_end, _ptr(s)),
           "psa_ref_run_period")
    return s


def anneal_period(n, eu, ev, ej, h, i0, lam, off, period, t_res, seed, trial_begin, trial_end):
    """Period-mode anneal: initial spins, len(i0) cycles, energy and cut."""
    s0 = init_spins(n, seed, trial_begin, trial_end)
    s = run_period(n, eu, ev, ej, h, i0, lam, off, period, t_res, seed, trial_begin,
                   trial_end, 0, len(i0), s0)
    E, C = energy_cut(n, eu, ev, ej, h, s)
    return s, E, C


def run_tapsa(n, eu, ev, ej, h, i0, lam, off, thr, alpha, seed, trial_begin, trial_end,
              t_begin, t_end, spins, ring=None):
    """TApSA sweeps t_begin..t_end-1 (Eq. 4) on copies of `spins` and of the
    field windows `ring` ([trials][n][alpha] int32; needed when t_begin > 0).
    Returns (spins, ring)."""
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    i0 = np.ascontiguousarray(i0, dtype=np.float32)
    lam = np.ascontiguousarray(lam, dtype=np.float32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    if i0.size < t_end or lam.size != n or off.size != n or thr.size != n:
        raise ValueError("schedule or per-p-bit arrays have the wrong size")
    rows = trial_end - trial_begin
    s = np.ascontiguousarray(np.array(spins, dtype=np.int8, copy=True).reshape(rows, n))
    if ring is None:
        if t_begin > 0:
            raise ValueError("ring is needed to resume at t_begin > 0")
        rg = np.zeros((rows, n, alpha), np.int32)
    else:
        rg = np.ascontiguousarray(np.array(ring, dtype=np.int32, copy=True).reshape(rows, n, alpha))
    _check(_load().psa_ref_run_tapsa(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej), _ptr(h),
                                     _ptr(i0), _ptr(lam), _ptr(off), _ptr(thr), int(alpha),
                                     seed, trial_begin, trial_end, t_begin, t_end, _ptr(s),
                                     _ptr(rg)),
           "psa_ref_run_tapsa")
    return s, rg


def anneal_tapsa(n, eu, ev, ej, h, i0, lam, off, thr, alpha, seed, trial_begin, trial_end):
    """TApSA anneal: initial spins, len(i0) sweeps, energy and cut per trial."""
    s0 = init_spins(n, seed, trial_begin, trial_end)
    s, _ = run_tapsa(n, eu, ev, ej, h, i0, lam, off, thr, alpha, seed, trial_begin,
                     trial_end, 0, len(i0), s0)
    E, C = energy_cut(n, eu, ev, ej, h, s)
    return s, E, C


def anneal_spsa(n, eu, ev, ej, h, i0, lam, off, thr, stall24, seed, trial_begin, trial_end):
    """SpSA anneal: initial spins, len(i0) sweeps, energy and cut per trial."""
    s0 = init_spins(n, seed, trial_begin, trial_end)
    s, _ = run_spsa(n, eu, ev, ej, h, i0, lam, off, thr, stall24, seed, trial_begin,
                    trial_end, 0, len(i0), s0)
    E, C = energy_cut(n, eu, ev, ej, h, s)
    return s, E, C


def energy_cut(n, eu, ev, ej, h, spins):
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    spins = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1, n)
    E = np.zeros(spins.shape[0], np.int64)
    C = np.zeros(spins.shape[0], np.int64)
    _check(_load().psa_ref_energy_cut(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej),
                                      _ptr(h), spins.shape[0], _ptr(spins),
                                      _ptr(E), _ptr(C)), "psa_ref_energy_cut")
    return E, C


def anneal(n, eu, ev, ej, h, i0, lam, off, thr, seed, trial_begin, trial_end):
    """Initial spins, len(i0) sweeps, then energy and cut per trial."""
    eu, ev, ej = _edges(eu, ev, ej)
    h = _opt_h(h, n)
    i0 = np.ascontiguousarray(i0, dtype=np.float32)
    lam = np.ascontiguousarray(lam, dtype=np.float32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    rows = trial_end - trial_begin
    spins = np.zeros((rows, n), np.int8)
    E = np.zeros(rows, np.int64)
    C = np.zeros(rows, np.int64)
    _check(_load().psa_ref_anneal(n, eu.size, _ptr(eu), _ptr(ev), _ptr(ej),
                                  _ptr(h), i0.size, _ptr(i0), _ptr(lam),
                                  _ptr(off), _ptr(thr), seed, trial_begin,
                                  trial_end, _ptr(spins), _ptr(E), _ptr(C)),
           "psa_ref_anneal")
    return spins, E, C


def anneal_parallel(n, eu, ev, ej, h, i0, lam, off, thr, seed, trials,
                    workers=None):
    """The same anneal with the trials split over host threads.

    Trials are independent and their random words are addressed by the
    trial index, so any split gives the same result as one call.
    """
    from concurrent.futures import ThreadPoolExecutor
    workers = workers or min(os.cpu_count() or 1, 16)
    bounds = np.linspace(0, trials, min(workers, trials) + 1).astype(int)
    parts = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with ThreadPoolExecutor(len(parts)) as ex:
        res = list(ex.map(lambda ab: anneal(n, eu, ev, ej, h, i0, lam, off, thr,
                                            seed, ab[0], ab[1]), parts))
    spins = np.concatenate([r[0] for r in res])
    E = np.concatenate([r[1] for r in res])
    C = np.concatenate([r[2] for r in res])
    return spins, E, C
