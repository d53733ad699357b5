"""GPU parity at the full sizes of the batched and served workloads.

* The batched mix: 256 graphs, n in [800, 5000] (half G(n, p) with +1
  weights, half degree 4-8 with +-1 weights), 64 trials, 1,000 steps, every
  job's path and launch shape from the autotuner in batched mode, all jobs
  advanced by one batched launch sequence -- exactly as the benchmark runs
  it.  Sampled (job, trial) pairs of both path families and of the first,
  middle and last trial tiles are recomputed by the oracle and compared spin
  by spin; the energy and cut of every trial of every job are compared with
  the oracle's evaluation of the device spins.
* The served mix: jobs of the serving trace at its extremes (n up to
  20,000, degree up to 50, up to 10,000 steps, 32-256 trials, variability
  sigma 0, 0.05, 0.1 and 0.2) submitted together to a server with the
  autotuner on; sampled trials against the oracle, every trial's energy and
  cut against the oracle's evaluation of the served spins.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


def _oracle_trial(n, u, v, w, steps, seed, sig, k):
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, steps)
    lam, dlt, thr = oracle.variability(n, seed, *sig)
    return oracle.anneal(n, u, v, -w, None, i0, lam, dlt, thr, seed, k, k + 1)


def test_batched_mix_256_graphs_sampled_against_oracle(psa):
    t0 = time.perf_counter()
    specs = inputs.batch_jobs(256)
    graphs_np = [inputs.make_graph(sp["graph"]) for sp in specs]
    _say(f"[c4] {len(specs)} graphs generated in {time.perf_counter() - t0:.1f} s")
    ctx = psa.Context(0)
    graphs, jobs = [], []
    for sp, (n, u, v, w) in zip(specs, graphs_np):
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        rb = psa.tune_get(ctx, g, sp["steps"], sp["trials"], sp["seed"], batch=True)
        kb = psa.tune_kwargs(rb)
        if kb["trials_per_group"] == 0:
            kb["trials_per_group"] = 1
        jobs.append(psa.Job(ctx, g, sp["steps"], sp["trials"], sp["seed"], **kb))
        graphs.append(g)
    dense = [j.dense for j in jobs]
    _say(f"[c4] tuned and created in {time.perf_counter() - t0:.1f} s: "
         f"{sum(dense)} dense, {len(jobs) - sum(dense)} CSR, "
         f"{psa.tune_cache_size(ctx)} shape classes")
    assert 0 < sum(dense) < len(jobs), "both path families must be in the mix"
    S = specs[0]["steps"]
    psa.jobs_step_batch(ctx, jobs, S)
    spins = [j.read_spins() for j in jobs]
    ec = [j.energy_cut() for j in jobs]
    _say(f"[c4] batched anneal done at {time.perf_counter() - t0:.1f} s")

    # sampled pairs: the largest, smallest and two further jobs of each family,
    # each at a first-tile and a last-tile (or middle) trial
    def pick(family):
        idx = [i for i in range(len(jobs)) if dense[i] == family]
        by_n = sorted(idx, key=lambda i: graphs_np[i][0])
        return [by_n[-1], by_n[0], by_n[len(by_n) // 3], by_n[(2 * len(by_n)) // 3]]

    pairs = []
    for family in (True, False):
        for r, gi in enumerate(pick(family)):
            pairs += [(gi, 0 if r % 2 == 0 else 17), (gi, 63 if r % 2 == 0 else 31)]
    assert len(pairs) == 16
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(lambda p: _oracle_trial(*graphs_np[p[0]], S, specs[p[0]]["seed"],
                                                  (0.0, 0.0, 0.0, 1.0), p[1]), pairs))
    for (gi, k), (os_, oE, oC) in zip(pairs, res):
        np.testing.assert_array_equal(spins[gi][k], os_[0],
                                      err_msg=f"job {gi} (dense={dense[gi]}) trial {k}")
        assert ec[gi][0][k] == oE[0] and ec[gi][1][k] == oC[0], (gi, k)
    _say(f"[c4] {len(pairs)} sampled trials equal the oracle at {time.perf_counter() - t0:.1f} s")

    def check_all(gi):
        n, u, v, w = graphs_np[gi]
        E, C = oracle.energy_cut(n, u, v, -w, None, spins[gi])
        return np.array_equal(E, ec[gi][0]) and np.array_equal(C, ec[gi][1])

    with ThreadPoolExecutor(16) as ex:
        ok = list(ex.map(check_all, range(len(jobs))))
    assert all(ok), [i for i, o in enumerate(ok) if not o][:10]
    for j in jobs:
        j.close()
    for g in graphs:
        g.close()
    ctx.close()


def _served_sample():
    """Jobs of the 50 jobs/s x 120 s serving trace at its extremes: the
    largest n, the most steps, the densest graph and the largest trial count,
    plus one job of every sigma, without repeats."""
    trace = [sp for _, sp in inputs.serve_trace(rate=50.0, duration=120.0)]
    def deg(sp):
        return 2 * sp["graph"][2] / sp["graph"][1]
    # bound the oracle's work (n x degree x steps per trial) for the ordinary picks
    cost = lambda sp: sp["graph"][1] * deg(sp) * sp["steps"]
    chosen = []
    for key in (lambda sp: sp["graph"][1], lambda sp: sp["steps"], deg, lambda sp: sp["trials"]):
        best = max((sp for sp in trace if cost(sp) < 4e9), key=key)
        if best not in chosen:
            chosen.append(best)
    for sigma in (0.0, 0.05, 0.1, 0.2):
        if not any(sp["sigma_nu"] == sigma for sp in chosen):
            chosen.append(next(sp for sp in trace if sp["sigma_nu"] == sigma and cost(sp) < 2e9))
    return chosen


def test_served_mix_at_full_sizes_against_oracle(psa):
    t0 = time.perf_counter()
    chosen = _served_sample()
    assert max(sp["graph"][1] for sp in chosen) >= 19000
    assert max(sp["steps"] for sp in chosen) >= 9500
    assert {sp["sigma_nu"] for sp in chosen} == {0.0, 0.05, 0.1, 0.2}
    graphs_np = [inputs.make_graph(sp["graph"]) for sp in chosen]
    for sp, (n, u, v, w) in zip(chosen, graphs_np):
        _say(f"[c5] job {sp['seed']}: n={n} edges={u.size} steps={sp['steps']} "
             f"trials={sp['trials']} sigma={sp['sigma_nu']}")
    ctx = psa.Context(0)
    srv = psa.Server(ctx, quantum_steps=250, max_resident=128)
    tickets = []
    for sp, (n, u, v, w) in zip(chosen, graphs_np):
        tickets.append(srv.submit(n, u, v, w, sp["steps"], sp["trials"], sp["seed"], spins=True,
                                  sigma_lambda=sp["sigma_lambda"], sigma_delta=sp["sigma_delta"],
                                  sigma_nu=sp["sigma_nu"], p_mean=sp["p_mean"], tune=True))
    results = [srv.result(t) for t in tickets]
    st = srv.stats()
    srv.close()
    _say(f"[c5] served {st['completed']} jobs in {time.perf_counter() - t0:.1f} s")
    assert st["completed"] == len(chosen) and st["failed"] == 0
    work = []
    for idx, (sp, (r, _)) in enumerate(zip(chosen, results)):
        assert r.status == psa.PSA_JOB_DONE
        assert r.submit_us <= r.admit_us <= r.start_us <= r.end_us
        T = sp["trials"]
        ks = [0, T - 1] if idx > 0 else [T // 2]
        work += [(idx, k) for k in ks]

    def ref(p):
        idx, k = p
        sp = chosen[idx]
        sig = (sp["sigma_lambda"], sp["sigma_delta"], sp["sigma_nu"], sp["p_mean"])
        return _oracle_trial(*graphs_np[idx], sp["steps"], sp["seed"], sig, k)

    with ThreadPoolExecutor(min(16, len(work))) as ex:
        res = list(ex.map(ref, work))
    for (idx, k), (os_, oE, oC) in zip(work, res):
        S_, E, C = results[idx][1]
        np.testing.assert_array_equal(S_[k], os_[0], err_msg=f"served job {idx} trial {k}")
        assert E[k] == oE[0] and C[k] == oC[0]
    for idx, (n, u, v, w) in enumerate(graphs_np):
        S_, E, C = results[idx][1]
        oE, oC = oracle.energy_cut(n, u, v, -w, None, S_)
        np.testing.assert_array_equal(E, oE)
        np.testing.assert_array_equal(C, oC)
    _say(f"[c5] {len(work)} sampled trials equal the oracle at {time.perf_counter() - t0:.1f} s")
    ctx.close()
