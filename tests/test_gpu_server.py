"""GPU tests of the serving loop: results served in a mix equal the same runs
alone; admission respects the HBM budget and slot cap; cancel, time-outs and
a failing request are handled without disturbing the other jobs.  Failure
conditions are forced from the host (tiny budgets, bad graphs, cancels)."""
import time

import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


def _alone(psa, ctx, spec):
    (n, u, v, w), T, S, seed, sig = spec
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    out = psa.anneal(ctx, g, S, T, seed, sigma_lambda=sig[0], sigma_delta=sig[1],
                     sigma_nu=sig[2], p_mean=sig[3])
    g.close()
    return out


def _specs():
    return [
        (inputs.gnm(700, 2100, 1), 6, 90, 31, (0.1, 0.1, 0.1, 0.8)),
        (inputs.erdos_renyi(300, 0.05, 2), 3, 40, 32, (0.0, 0.0, 0.0, 1.0)),
        (inputs.torus(10, 30, 3), 12, 120, 33, (0.2, 0.05, 0.1, 0.8)),
        (inputs.gnm(1500, 6000, 4), 2, 65, 34, (0.05, 0.05, 0.05, 0.8)),
        (inputs.gnm(64, 300, 5), 40, 33, 35, (0.0, 0.0, 0.0, 1.0)),
        (inputs.gnm(2500, 9000, 6), 5, 150, 36, (0.1, 0.1, 0.1, 0.8)),
    ]


def _submit(srv, spec, spins=True, **kw):
    (n, u, v, w), T, S, seed, sig = spec
    return srv.submit(n, u, v, w, S, T, seed, spins=spins, sigma_lambda=sig[0],
                      sigma_delta=sig[1], sigma_nu=sig[2], p_mean=sig[3], **kw)


def test_served_results_equal_alone(psa):
    """Staggered arrivals, quantum 17 steps, at most 3 resident: jobs overlap
    on the device and join as slots free up; every result equals its run
    alone, and one equals the oracle."""
    ctx = psa.Context(0)
    specs = _specs()
    ref = [_alone(psa, ctx, sp) for sp in specs]
    srv = psa.Server(ctx, max_resident=3, quantum_steps=17)
    tickets = []
    for sp in specs:
        tickets.append(_submit(srv, sp))
        time.sleep(0.002)
    results = [srv.result(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(specs) and st["failed"] == 0
    for (r, (S, E, C)), (rS, rE, rC) in zip(results, ref):
        assert r.status == psa.PSA_JOB_DONE
        np.testing.assert_array_equal(S, rS)
        np.testing.assert_array_equal(E, rE)
        np.testing.assert_array_equal(C, rC)
        assert r.submit_us <= r.admit_us <= r.start_us <= r.end_us
    (n, u, v, w), T, S_, seed, sig = specs[2]
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, S_)
    lam, dl, thr = oracle.variability(n, seed, *sig)
    o = oracle.anneal(n, u, v, -w, None, i0, lam, dl, thr, seed, 0, T)
    np.testing.assert_array_equal(results[2][1][0], o[0])
    ctx.close()


def test_budget_serialises_and_rejects(psa):
    ctx = psa.Context(0)
    specs = _specs()[:3]
    # a budget of about one of these jobs: they queue for memory (the CSR path
    # is forced, so that no dense matrix is reserved for them)
    budget = 150_000
    srv = psa.Server(ctx, hbm_budget_bytes=budget, quantum_steps=25)
    tickets = [_submit(srv, sp, spins=False, path=psa.PSA_PATH_CSR) for sp in specs]
    big = srv.submit(*inputs.gnm(20000, 60000, 9), 10, 200, 1)      # alone above budget
    while True:
        st = srv.stats()
        if st["completed"] + st["failed"] >= 4:
            break
        time.sleep(0.001)
    for t, sp in zip(tickets, specs):
        r, (_, E, C) = srv.result(t)
        assert r.status == psa.PSA_JOB_DONE
        np.testing.assert_array_equal(C, _alone(psa, ctx, sp)[2])
    r = srv.wait(big)
    assert r.status == psa.PSA_JOB_ERROR and r.error == psa.PSA_ENOMEM
    assert 1 <= st["peak_resident"] < 3 and 0 < st["peak_used_bytes"] <= budget
    srv.close()
    ctx.close()


def test_cancel_timeout_and_bad_request(psa):
    ctx = psa.Context(0)
    srv = psa.Server(ctx, quantum_steps=50)
    n, u, v, w = inputs.gnm(3000, 12000, 7)
    long_job = srv.submit(n, u, v, w, 100000, 64, 3)
    bad = srv.submit(3, np.array([0, 1]), np.array([0, 2]), np.array([1, 1]), 10, 2, 0)
    ok_spec = _specs()[1]
    ok = _submit(srv, ok_spec)
    with pytest.raises(psa.PsaError) as e:
        srv.wait(long_job, timeout_s=0.05)
    assert e.value.status == psa.PSA_ETIMEDOUT
    srv.cancel(long_job)
    assert srv.wait(long_job).status == psa.PSA_JOB_CANCELED
    r = srv.wait(bad)
    assert r.status == psa.PSA_JOB_ERROR and r.error == psa.PSA_EINVAL
    r, (S, E, C) = srv.result(ok)
    assert r.status == psa.PSA_JOB_DONE
    np.testing.assert_array_equal(S, _alone(psa, ctx, ok_spec)[0])
    srv.close()
    ctx.close()


def _wait_for(cond, what, limit_s=30.0):
    t0 = time.perf_counter()
    while not cond():
        if time.perf_counter() - t0 > limit_s:
            raise AssertionError(f"timed out waiting for {what}")
        time.sleep(0.001)


def test_queue_limit_returns_eagain(psa):
    """max_waiting = 2: with one long job resident (one slot), two more wait
    and the next submission is refused with PSA_EAGAIN until one is admitted."""
    ctx = psa.Context(0)
    srv = psa.Server(ctx, max_resident=1, quantum_steps=50, max_waiting=2)
    n, u, v, w = inputs.gnm(2000, 6000, 21)
    long_job = srv.submit(n, u, v, w, 1_000_000, 32, 1)
    _wait_for(lambda: srv.stats()["resident"] == 1, "the long job to be admitted")
    small = _specs()[4]
    queued = [_submit(srv, small, spins=False), _submit(srv, small, spins=False)]
    with pytest.raises(psa.PsaError) as e:
        _submit(srv, small, spins=False)
    assert e.value.status == psa.PSA_EAGAIN
    assert srv.stats()["waiting"] == 2
    srv.cancel(long_job)
    assert srv.wait(long_job).status == psa.PSA_JOB_CANCELED
    for t in queued:                       # admitted once the slot frees up
        assert srv.wait(t).status == psa.PSA_JOB_DONE
    later = _submit(srv, small, spins=False)
    assert srv.wait(later).status == psa.PSA_JOB_DONE
    srv.close()
    ctx.close()


def test_dense_job_footprint_counts_its_matrix(psa):
    """A served dense-path job is charged what it holds on the device: its
    graph with the dense coupling matrix, its dense spin buffers and run state
    (the same allocations as the job created alone), plus read-out staging."""
    n, u, v, w = inputs.erdos_renyi(3000, 0.08, 31)
    T = 64
    ctx = psa.Context(0)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    alone = psa.Job(ctx, g, 100_000, T, 2, path=psa.PSA_PATH_DENSE)
    assert alone.dense
    held = g.info()["device_bytes"] + alone.info()["device_bytes"]
    np_ = (n + 127) // 128 * 128
    assert g.info()["device_bytes"] >= np_ * np_ // 4           # the 2-bit matrix
    alone.close()
    g.close()
    srv = psa.Server(ctx, quantum_steps=50)
    t = srv.submit(n, u, v, w, 100_000, T, 2, path=psa.PSA_PATH_DENSE)
    _wait_for(lambda: srv.stats()["resident"] == 1, "the dense job to be admitted")
    used = srv.stats()["used_bytes"]
    assert held <= used <= held + (1 << 20), (held, used)
    srv.cancel(t)
    assert srv.wait(t).status == psa.PSA_JOB_CANCELED
    assert srv.stats()["used_bytes"] == 0
    srv.close()
    ctx.close()
