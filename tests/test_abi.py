"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/psa.h declares, and its host-side logic (schedule, variability draw)
matches the oracle bit for bit.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psa.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(psa_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


def test_library_exports_every_declared_symbol(psa):
    lib = ctypes.CDLL(psa.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows each of them under the same name
    assert sorted(psa.EXPORTED) == declared


def test_version_and_error_text(psa):
    assert "gfx950" in psa.version()
    assert psa.psa_last_error() is not None


@pytest.mark.parametrize("steps,lo,hi", [(1000, 0.0149880307, 1.49880307),
                                         (5000, 0.05, 5.0), (2, 0.3, 0.3), (1, 0.2, 9.0),
                                         (2000, 1e-3, 1e3)])
def test_schedule_fill_matches_oracle(psa, steps, lo, hi):
    np.testing.assert_array_equal(psa.schedule_fill(steps, lo, hi),
                                  oracle.schedule(steps, lo, hi))


def test_schedule_rejects_bad_endpoints(psa):
    with pytest.raises(psa.PsaError) as e:
        psa.schedule_fill(10, 0.0, 1.0)
    assert e.value.status == psa.PSA_EINVAL
    with pytest.raises(psa.PsaError):
        psa.schedule_fill(0, 0.1, 1.0)


@pytest.mark.parametrize("sig", [(0.0, 0.0, 0.0, 1.0), (0.1, 0.1, 0.1, 0.8),
                                 (0.2, 0.05, 1.0, 0.5), (0.0, 0.0, 0.3, 0.0)])
def test_variability_draw_matches_oracle(psa, sig):
    for seed in (0, 3, 2**63 + 12345):
        got = psa.variability_draw(5000, seed, *sig)
        ref = oracle.variability(5000, seed, *sig)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("sig,t_res", [(0.0, 10), (0.1, 10), (0.3, 7), (2.0, 10), (0.2, 1)])
def test_periods_draw_matches_oracle(psa, sig, t_res):
    for seed in (0, 5, 2**63 + 7):
        np.testing.assert_array_equal(psa.periods_draw(5000, seed, sig, t_res),
                                      oracle.periods(5000, seed, sig, t_res))
    with pytest.raises(psa.PsaError):
        psa.periods_draw(10, 0, sig, 0)


def test_variability_rejects_bad_parameters(psa):
    with pytest.raises(psa.PsaError):
        psa.variability_draw(10, 0, -0.1, 0, 0, 1)
    with pytest.raises(psa.PsaError):
        psa.variability_draw(10, 0, 0, 0, 0, 1.5)


def test_binding_has_no_cpu_path():
    """The binding module holds no update arithmetic: no tanh, no Philox."""
    src = open(os.path.join(ROOT, "paper_2601_14476_amd", "psa.py")).read()
    for word in ("philox", "0xd2511f53", "import oracle", "from oracle", "np.tanh",
                 "math.tanh", "torch.tanh"):
        assert word not in src.lower(), word


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_graph_check_edges_matches_oracle(psa, name):
    """Host-side ingestion statistics (no device): counts, W_total and the
    paper's mean(s_i) against the oracle, degree bound from the edge list."""
    from paper_2601_14476_amd import inputs
    spec = inputs.workload(name)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    info = psa.graph_check_edges(n, u, v, w)
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    assert info["n"] == n and info["edges"] == u.size and info["nnz"] == 2 * u.size
    assert info["w_total"] == int(w.sum())
    assert info["max_degree"] == int(deg.max())
    assert info["max_abs_field"] == int(deg.max())
    assert info["unit_weights"] == 1 and info["device_bytes"] == 0
    assert info["mean_s"] == oracle.mean_s(n, u, v, -w)


def test_graph_check_edges_rejects_invalid_graphs(psa):
    z = np.array([0], np.int32)
    o = np.array([1], np.int32)
    cases = [(2, z, z, o),                                        # self loop
             (2, np.array([0, 1], np.int32), np.array([1, 0], np.int32),
              np.array([1, 1], np.int32)),                        # repeated pair
             (2, z, np.array([5], np.int32), o),                  # out of range
             (2, z, o, np.array([1 << 24], np.int32))]            # field bound 2^24
    for n, u, v, w in cases:
        with pytest.raises(psa.PsaError) as e:
            psa.graph_check_edges(n, u, v, w)
        assert e.value.status == psa.PSA_EINVAL


_ENOMEM_CHILD = r"""
import ctypes, resource, sys
import numpy as np

class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("edges", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("w_total", ctypes.c_int64), ("max_abs_field", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("unit_weights", ctypes.c_int32),
                ("mean_s", ctypes.c_double), ("device_bytes", ctypes.c_int64)]

lib = ctypes.CDLL(sys.argv[1])
lib.psa_last_error.restype = ctypes.c_char_p
ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
# a valid circulant graph: p-bit i joined to i+1 .. i+15 (mod n), 30 M edges
n, K = 2_000_000, 15
u = np.repeat(np.arange(n, dtype=np.int32), K)
v = ((u.astype(np.int64) + np.tile(np.arange(1, K + 1), n)) % n).astype(np.int32)
w = np.ones(u.size, np.int32)
info = Info()
# room for the library's first arrays but not for the CSR (240 MB per array)
vm = int(open("/proc/self/status").read().split("VmSize:")[1].split()[0]) * 1024
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
resource.setrlimit(resource.RLIMIT_AS, (vm + (64 << 20), hard))
st = lib.psa_graph_check_edges(n, u.size, ptr(u), ptr(v), ptr(w), None, 1, ctypes.byref(info))
msg = lib.psa_last_error().decode()
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
# the library is still usable afterwards
u2, v2, w2 = np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.ones(2, np.int32)
st2 = lib.psa_graph_check_edges(3, 2, ptr(u2), ptr(v2), ptr(w2), None, 1, ctypes.byref(info))
print(st, st2, info.edges, msg)
"""


def test_host_allocation_failure_is_a_status_not_a_crash(psa):
    """A failed host allocation inside an exported call returns PSA_ENOMEM
    with an error text, instead of an exception unwinding through the C ABI
    (which would abort the process).  Forced in a child process by capping
    its address space just above what it has mapped."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, "-c", _ENOMEM_CHILD, psa.LIB_PATH],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr[-2000:]
    st, st2, edges, *msg = res.stdout.split()
    assert int(st) == psa.PSA_ENOMEM, res.stdout
    assert "psa_graph_check_edges" in " ".join(msg) and "allocation" in " ".join(msg)
    assert int(st2) == psa.PSA_OK and int(edges) == 2


def test_batched_calls_reject_a_null_context_on_the_host(psa):
    """The batched step and read-out check their arguments before any device
    call: a NULL context (with or without jobs, with a negative count or
    unknown flags) is EINVAL with an error text naming the call, and an
    empty list on a NULL context is still an error."""
    lib = psa._lib
    P = ctypes.c_void_p
    cases = [
        ("psa_jobs_energy_cut", lambda: lib.psa_jobs_energy_cut(None, 0, None, None, None, 0)),
        ("psa_jobs_energy_cut", lambda: lib.psa_jobs_energy_cut(None, -1, None, None, None, 0)),
        ("psa_jobs_energy_cut", lambda: lib.psa_jobs_energy_cut(None, 0, None, None, None, 0x80)),
        ("psa_jobs_energy_cut", lambda: lib.psa_jobs_energy_cut(
            None, 1, (P * 1)(None), (P * 1)(None), (P * 1)(None), 0)),
        ("psa_jobs_step_batch", lambda: lib.psa_jobs_step_batch(None, 0, None, 1)),
        ("psa_jobs_step_batch", lambda: lib.psa_jobs_step_batch(None, 1, (P * 1)(None), 1)),
    ]
    for name, call in cases:
        assert call() == psa.PSA_EINVAL, name
        assert name in lib.psa_last_error().decode()
