"""GPU parity of the batched launch: many graphs of uneven size and weight
type in one launch give exactly the results of running each alone, and of
the oracle; jobs advanced in step quanta, with a job joining mid-way, end
where a single uninterrupted run ends."""
import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


@pytest.fixture(scope="module")
def ctx(psa):
    c = psa.Context(0)
    yield c
    c.close()


def _mix():
    """(n, u, v, J, h, maxcut_w or None, trials, steps, seed, sigmas) of a mixed batch."""
    rng = np.random.default_rng(3)
    out = []
    for idx, (kind, n, trials, steps) in enumerate([
            ("er1", 300, 8, 40), ("gnm", 811, 3, 55), ("torus", 0, 10, 30), ("int", 257, 5, 25),
            ("big", 97, 4, 20), ("gnm", 2000, 33, 12), ("er1", 1203, 1, 35), ("int", 64, 7, 60),
            ("gnm", 5, 2, 15), ("hub", 400, 6, 18)]):
        if kind == "er1":
            n, u, v, w = inputs.erdos_renyi(n, 0.05, 100 + idx)
            j, h = -w, None
        elif kind == "gnm":
            n, u, v, w = inputs.gnm(n, min(3 * n, n * (n - 1) // 2), 100 + idx)
            j, h = -w, None
        elif kind == "torus":
            n, u, v, w = inputs.torus(12, 15, 100 + idx)
            j, h = -w, None
        elif kind == "hub":
            hub = np.arange(1, 301, dtype=np.int32)
            ring_u = np.arange(1, n, dtype=np.int32)
            ring_v = np.roll(ring_u, -1)
            u = np.concatenate([np.zeros(300, np.int32), np.minimum(ring_u, ring_v)])
            v = np.concatenate([hub, np.maximum(ring_u, ring_v)])
            j = rng.choice([-1, 1], size=u.size).astype(np.int32)
            h = None
        else:
            _, u, v, _ = inputs.gnm(n, 3 * n, 100 + idx)
            jmax = 4 if kind == "int" else 3
            j = (rng.integers(1, jmax + 1, size=u.size) * rng.choice([-1, 1], size=u.size))
            h = rng.integers(-5, 6, size=n)
            if kind == "big":
                j = j * 15000
                h = h * 2000
            j = j.astype(np.int32)
            h = h.astype(np.int32)
        sig = (0.1, 0.1, 0.1, 0.8) if idx % 2 == 0 else (0.0, 0.0, 0.0, 1.0)
        out.append((n, u, v, j, h, trials, steps, 1000 + idx, sig))
    return out


def _schedule(kind_big, steps):
    return oracle.schedule(steps, 1e-5, 1e-4) if kind_big else oracle.schedule(steps, 0.02, 0.8)


def test_batch_equals_sequential_and_oracle(psa, ctx):
    mix = _mix()
    graphs, items = [], []
    for n, u, v, j, h, T, S, seed, sig in mix:
        g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
        graphs.append(g)
        i0 = _schedule(int(np.abs(j).max()) > 1000, S)
        items.append((g, S, T, seed, dict(i0=i0, sigma_lambda=sig[0], sigma_delta=sig[1],
                                          sigma_nu=sig[2], p_mean=sig[3])))
    batched = psa.anneal_batch(ctx, items, spins=True)
    seq = psa.anneal_batch(ctx, items, sequential=True, spins=True)
    for (bs, bE, bC), (ss, sE, sC) in zip(batched, seq):
        np.testing.assert_array_equal(bs, ss)
        np.testing.assert_array_equal(bE, sE)
        np.testing.assert_array_equal(bC, sC)
    for (n, u, v, j, h, T, S, seed, sig), (bs, bE, bC) in zip(mix, batched):
        i0 = _schedule(int(np.abs(j).max()) > 1000, S)
        lam, dl, thr = oracle.variability(n, seed, *sig)
        k = min(T, 2)
        ref = oracle.anneal(n, u, v, j, h, i0, lam, dl, thr, seed, 0, k)
        np.testing.assert_array_equal(bs[:k], ref[0])
        np.testing.assert_array_equal(bE[:k], ref[1])
        np.testing.assert_array_equal(bC[:k], ref[2])


def test_step_quanta_with_late_joiner(psa, ctx):
    """Continuous batching semantics: jobs advance together in quanta of 7
    steps; a job created after three quanta joins the next launches.  Every
    job ends exactly where an uninterrupted single run ends."""
    specs = [(inputs.gnm(500, 1500, 7), 5, 40, 11, (0.1, 0.1, 0.1, 0.8)),
             (inputs.erdos_renyi(350, 0.04, 8), 9, 23, 12, (0.0, 0.0, 0.0, 1.0)),
             (inputs.torus(10, 20, 9), 4, 31, 13, (0.2, 0.05, 0.2, 0.7))]
    late = (inputs.gnm(901, 2700, 10), 6, 26, 14, (0.05, 0.05, 0.05, 0.8))

    def make(spec):
        (n, u, v, w), T, S, seed, sig = spec
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        job = psa.Job(ctx, g, S, T, seed, sigma_lambda=sig[0], sigma_delta=sig[1],
                      sigma_nu=sig[2], p_mean=sig[3])
        ref = psa.Job(ctx, g, S, T, seed, sigma_lambda=sig[0], sigma_delta=sig[1],
                      sigma_nu=sig[2], p_mean=sig[3])
        ref.step(S)
        return g, job, ref

    live = [make(s) for s in specs]
    rounds = 0
    while any(j.position < j.steps for _, j, _ in live):
        psa.jobs_step_batch(ctx, [j for _, j, _ in live if j.position < j.steps], 7)
        rounds += 1
        if rounds == 3:
            live.append(make(late))
    for g, job, ref in live:
        assert job.position == job.steps
        np.testing.assert_array_equal(job.read_spins(), ref.read_spins())
        np.testing.assert_array_equal(job.energy_cut()[1], ref.energy_cut()[1])
    # and one of them against the oracle
    (n, u, v, w), T, S, seed, sig = specs[2]
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, S)
    lam, dl, thr = oracle.variability(n, seed, *sig)
    ref = oracle.anneal(n, u, v, -w, None, i0, lam, dl, thr, seed, 0, T)
    np.testing.assert_array_equal(live[2][1].read_spins(), ref[0])


def test_batch_rejects_bad_input(psa, ctx):
    n, u, v, w = inputs.gnm(50, 100, 1)
    g = psa.Graph.from_edges(ctx, n, u, v, w)
    job = psa.Job(ctx, g, 10, 2, 0)
    with pytest.raises(psa.PsaError):
        psa.jobs_step_batch(ctx, [job, job], 3)        # listed twice
    with pytest.raises(psa.PsaError):
        psa.anneal_batch(ctx, [(g, 0, 2, 0, {})])       # steps < 1


def test_batch_mixes_dense_and_csr_jobs(psa, ctx):
    """Dense-path and CSR-path jobs advanced together give the results of
    each alone."""
    specs = [(inputs.erdos_renyi(700, 0.2, 51), psa.PSA_PATH_DENSE, 64, 30),
             (inputs.gnm(900, 2700, 52), psa.PSA_PATH_CSR, 10, 45),
             (inputs.erdos_renyi(200, 0.5, 53), psa.PSA_PATH_DENSE, 20, 38),
             (inputs.torus(8, 9, 54), psa.PSA_PATH_AUTO, 3, 12)]
    # integer couplings |J| <= 4: the int8 encoding, in the same batch as 2-bit ones
    rng = np.random.default_rng(55)
    _, iu, iv, _ = inputs.gnm(450, 20000, 55)
    iw = (rng.integers(1, 5, size=iu.size) * rng.choice([-1, 1], size=iu.size)).astype(np.int32)
    specs.append(((450, iu, iv, iw), psa.PSA_PATH_DENSE, 17, 26))
    jobs, refs = [], []
    for (n, u, v, w), path, T, S in specs:
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        jobs.append(psa.Job(ctx, g, S, T, 5, path=path, sigma_nu=0.1, p_mean=0.8))
        ref = psa.Job(ctx, g, S, T, 5, path=psa.PSA_PATH_CSR, sigma_nu=0.1, p_mean=0.8)
        ref.step(S)
        refs.append(ref)
    while any(j.position < j.steps for j in jobs):
        psa.jobs_step_batch(ctx, [j for j in jobs if j.position < j.steps], 11)
    for j, r in zip(jobs, refs):
        np.testing.assert_array_equal(j.read_spins(), r.read_spins())
        np.testing.assert_array_equal(j.energy_cut()[0], r.energy_cut()[0])


def test_batch_four_trial_groups(psa, ctx):
    """Jobs with four trials per workgroup inside a batched launch (16-bit
    and 32-bit packed edges, column/value pairs, edges in LDS and in global
    memory), mixed with one-trial jobs: each ends where it ends alone."""
    rng = np.random.default_rng(71)
    specs = []
    n, u, v, w = inputs.gnm(700, 2100, 71)                       # +-1, LDS
    specs.append((n, u, v, -w, None, 4, 13, 40))
    n, u, v, w = inputs.gnm(6000, 60000, 72)                     # +-1, edges beyond LDS
    specs.append((n, u, v, -w, None, 4, 9, 25))
    n, u, v, _ = inputs.gnm(500, 2000, 73)                       # |J| <= 4: 32-bit packing
    j = (rng.integers(1, 5, size=u.size) * rng.choice([-1, 1], size=u.size)).astype(np.int32)
    specs.append((n, u, v, j, rng.integers(-3, 4, size=n).astype(np.int32), 4, 6, 33))
    n, u, v, _ = inputs.gnm(300, 900, 74)                        # |J| >= 2^15: pairs
    j = (rng.choice([-1, 1], size=u.size) * 40000).astype(np.int32)
    specs.append((n, u, v, j, None, 4, 5, 21))
    n, u, v, w = inputs.gnm(800, 2400, 75)                       # one-trial job in the mix
    specs.append((n, u, v, -w, None, 1, 7, 30))
    jobs, refs = [], []
    for n, u, v, j, h, tpw, T, S in specs:
        g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
        big = int(np.abs(j).max()) > 1000
        i0 = oracle.schedule(S, 1e-5, 1e-4) if big else oracle.schedule(S, 0.02, 0.8)
        kw = dict(i0=i0, sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
        jobs.append(psa.Job(ctx, g, S, T, 9, trials_per_group=tpw, path=psa.PSA_PATH_CSR, **kw))
        ref = psa.Job(ctx, g, S, T, 9, trials_per_group=1, path=psa.PSA_PATH_CSR, **kw)
        ref.step(S)
        refs.append(ref)
    while any(jb.position < jb.steps for jb in jobs):
        psa.jobs_step_batch(ctx, [jb for jb in jobs if jb.position < jb.steps], 8)
    for jb, r in zip(jobs, refs):
        np.testing.assert_array_equal(jb.read_spins(), r.read_spins())
        np.testing.assert_array_equal(jb.energy_cut()[0], r.energy_cut()[0])


def test_batch_mixes_spsa_and_psa(psa, ctx):
    """SpSA, TApSA and pSA jobs on CSR (one and four trials per workgroup) and
    dense paths advance together in quanta and end where each ends alone."""
    specs = [(inputs.gnm(600, 1800, 95), psa.PSA_ALG_SPSA, psa.PSA_PATH_CSR, 1, 9, 33),
             (inputs.gnm(900, 2700, 96), psa.PSA_ALG_SPSA, psa.PSA_PATH_CSR, 4, 12, 27),
             (inputs.erdos_renyi(500, 0.2, 97), psa.PSA_ALG_SPSA, psa.PSA_PATH_DENSE, 0, 20, 31),
             (inputs.gnm(700, 2100, 98), psa.PSA_ALG_PSA, psa.PSA_PATH_CSR, 1, 5, 29),
             (inputs.gnm(650, 1950, 99), psa.PSA_ALG_TAPSA, psa.PSA_PATH_CSR, 1, 6, 25),
             (inputs.gnm(800, 2400, 100), psa.PSA_ALG_TAPSA, psa.PSA_PATH_CSR, 4, 10, 27),
             (inputs.erdos_renyi(450, 0.2, 101), psa.PSA_ALG_TAPSA, psa.PSA_PATH_DENSE, 0, 18, 22),
             # a pSA run in a dense list with other modes takes the general step
             (inputs.erdos_renyi(420, 0.2, 102), psa.PSA_ALG_PSA, psa.PSA_PATH_DENSE, 0, 13, 24)]
    kw = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8, p_stall=0.5, window=4)
    jobs, refs = [], []
    for (n, u, v, w), alg, path, tpw, T, S in specs:
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        jobs.append(psa.Job(ctx, g, S, T, 3, algorithm=alg, path=path, trials_per_group=tpw, **kw))
        ref = psa.Job(ctx, g, S, T, 3, algorithm=alg, path=psa.PSA_PATH_CSR, **kw)
        ref.step(S)
        refs.append(ref)
    while any(j.position < j.steps for j in jobs):
        psa.jobs_step_batch(ctx, [j for j in jobs if j.position < j.steps], 7)
    for j, r in zip(jobs, refs):
        np.testing.assert_array_equal(j.read_spins(), r.read_spins())


def test_dense_psa_list_with_a_period_run(psa, ctx):
    """Dense pSA runs alone use the step without mode tests; with a period-mode
    run in the same list, all of them take the general step.  Both end where
    each run ends alone on the CSR path."""
    kw = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
    graphs = [psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
              for n, u, v, w in (inputs.erdos_renyi(380, 0.25, 111), inputs.erdos_renyi(300, 0.3, 112))]
    for with_period in (False, True):
        jobs = [psa.Job(ctx, graphs[0], 21, 16, 5, path=psa.PSA_PATH_DENSE, **kw),
                psa.Job(ctx, graphs[1], 17, 9, 6, path=psa.PSA_PATH_DENSE, **kw)]
        refs = [psa.Job(ctx, graphs[0], 21, 16, 5, path=psa.PSA_PATH_CSR, **kw),
                psa.Job(ctx, graphs[1], 17, 9, 6, path=psa.PSA_PATH_CSR, **kw)]
        if with_period:
            jobs.append(psa.Job(ctx, graphs[1], 9, 5, 7, path=psa.PSA_PATH_DENSE, t_res=10, **kw))
            refs.append(psa.Job(ctx, graphs[1], 9, 5, 7, path=psa.PSA_PATH_CSR, t_res=10, **kw))
        for r in refs:
            r.step(r.steps)
        while any(j.position < j.steps for j in jobs):
            psa.jobs_step_batch(ctx, [j for j in jobs if j.position < j.steps], 6)
        for j, r in zip(jobs, refs):
            np.testing.assert_array_equal(j.read_spins(), r.read_spins())
            np.testing.assert_array_equal(j.energy_cut()[1], r.energy_cut()[1])


def test_dense_step_at_bench_size_sampled_trials(psa, ctx):
    """The dense matrix-core step at the size and in the launch the dense-step
    benchmark times: G(n, p) graphs with n in [2000, 4000] (one not a multiple
    of 128) and p in [0.04, 0.1], +1 weights (2-bit couplings), 64 trials, the
    paper's schedule over 1,000 steps, all runs in one dense list advanced in
    quanta.  Without variability the synchronous update of these dense
    antiferromagnetic couplings ends in the two uniform states (cut 0): the
    oscillation that the paper's variability breaks, and a full-size check of
    the same trajectory on both sides.  Sampled trials (first, middle, last of the trial tile) against
    the oracle; energy and cut of every trial against the oracle's evaluation
    of the device spins."""
    from concurrent.futures import ThreadPoolExecutor
    S, T = 1000, 64
    specs = [inputs.erdos_renyi(3968, 0.1, 700), inputs.erdos_renyi(2000, 0.04, 701),
             inputs.erdos_renyi(2777, 0.07, 702)]
    graphs = [psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True) for n, u, v, w in specs]
    # the second run also draws the three variability factors (gated updates)
    var = [(0.0, 0.0, 0.0, 1.0), (0.1, 0.1, 0.1, 0.8), (0.0, 0.0, 0.0, 1.0)]
    jobs = [psa.Job(ctx, g, S, T, 40 + i, path=psa.PSA_PATH_DENSE, sigma_lambda=var[i][0],
                    sigma_delta=var[i][1], sigma_nu=var[i][2], p_mean=var[i][3])
            for i, g in enumerate(graphs)]
    assert all(j.dense for j in jobs)
    for _ in range(4):
        psa.jobs_step_batch(ctx, jobs, S // 4)
    sample = [0, 31, 63]
    work = []
    for i, (n, u, v, w) in enumerate(specs):
        i0, _, _ = oracle.schedule_paper(n, u, v, -w, S)
        lam, dlt, thr = oracle.variability(n, 40 + i, *var[i])
        work += [(i, k, n, u, v, w, i0, lam, dlt, thr) for k in sample]
    with ThreadPoolExecutor(len(work)) as ex:
        res = list(ex.map(lambda a: oracle.anneal(a[2], a[3], a[4], -a[5], None, a[6], a[7], a[8], a[9],
                                                  40 + a[0], a[1], a[1] + 1), work))
    spins = [j.read_spins() for j in jobs]
    ec = [j.energy_cut() for j in jobs]
    for (i, k, *_), (os_, oE, oC) in zip(work, res):
        np.testing.assert_array_equal(spins[i][k], os_[0], err_msg=f"graph {i} trial {k}")
        assert ec[i][0][k] == oE[0] and ec[i][1][k] == oC[0]
    for i, (n, u, v, w) in enumerate(specs):
        E, C = oracle.energy_cut(n, u, v, -w, None, spins[i])
        np.testing.assert_array_equal(ec[i][0], E)
        np.testing.assert_array_equal(ec[i][1], C)


def test_dense_identity_list_against_oracle(psa, ctx):
    """A dense list whose runs all have identity factors and no timing gate
    takes the identity epilogue (pre-activation I0 (float)L, r blocks of the
    first eight row/trial pairs drawn during the matrix loop): graphs whose
    coupling chunks number fewer than eight (n = 700, 1,000) and more (n =
    2,300), 2-bit and int8 couplings, 64 and 40 trials, stepped in quanta;
    sampled trials against the oracle, energy and cut of every trial against
    the oracle's evaluation of the device spins."""
    S = 24
    rng = np.random.default_rng(90)
    specs = [inputs.erdos_renyi(700, 0.2, 91), inputs.erdos_renyi(2300, 0.05, 92)]
    n3, u3, v3, _ = inputs.erdos_renyi(1000, 0.1, 93)
    w3 = (rng.integers(1, 4, size=u3.size) * rng.choice([-1, 1], size=u3.size)).astype(np.int32)
    specs.append((n3, u3, v3, w3))
    trials = [64, 40, 64]
    graphs = [psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True) for n, u, v, w in specs]
    jobs = [psa.Job(ctx, g, S, T, 60 + i, path=psa.PSA_PATH_DENSE) for i, (g, T) in enumerate(zip(graphs, trials))]
    assert all(j.dense for j in jobs)
    for _ in range(3):
        psa.jobs_step_batch(ctx, jobs, S // 3)
    for i, ((n, u, v, w), T) in enumerate(zip(specs, trials)):
        i0, _, _ = oracle.schedule_paper(n, u, v, -w, S)
        lam, dlt, thr = oracle.variability(n, 60 + i, 0.0, 0.0, 0.0, 1.0)
        spins = jobs[i].read_spins()
        for k in (0, T // 2, T - 1):
            ref = oracle.anneal(n, u, v, -w, None, i0, lam, dlt, thr, 60 + i, k, k + 1)
            np.testing.assert_array_equal(spins[k], ref[0][0], err_msg=f"graph {i} trial {k}")
        E, C = oracle.energy_cut(n, u, v, -w, None, spins)
        got_E, got_C = jobs[i].energy_cut()
        np.testing.assert_array_equal(got_E, E)
        np.testing.assert_array_equal(got_C, C)


def test_jobs_energy_cut_matches_each_job_and_oracle(psa, ctx):
    """The batched energy / cut read-out of the mixed batch (uneven n and
    trial counts, integer and large couplings, fields h) plus dense-path
    jobs gives each job's own read-out, host and device outputs alike, and
    the oracle's energy and cut of the same spins (a job listed twice, an
    empty list)."""
    import torch
    mix = _mix()
    jobs, edges = [], []
    for n, u, v, j, h, T, S, seed, sig in mix:
        g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
        i0 = _schedule(int(np.abs(j).max()) > 1000, S)
        jobs.append(psa.Job(ctx, g, S, T, seed, i0=i0, sigma_lambda=sig[0], sigma_delta=sig[1],
                            sigma_nu=sig[2], p_mean=sig[3]))
        edges.append((n, u, v, j, h))
    for (n, u, v, w), T in [(inputs.erdos_renyi(700, 0.2, 61), 64), (inputs.erdos_renyi(300, 0.3, 62), 6)]:
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        jobs.append(psa.Job(ctx, g, 30, T, 7, path=psa.PSA_PATH_DENSE))
        edges.append((n, u, v, -w, None))
    # integer couplings and fields on rows of mean degree 30 and 93 (read by
    # 4 and 16 lanes a row), the second with large couplings
    rng = np.random.default_rng(64)
    for n, m, scale, T in [(200, 3000, 1, 20), (150, 7000, 30000, 16)]:
        _, u, v, _ = inputs.gnm(n, m, 64 + n)
        j = (rng.integers(1, 4, size=u.size) * rng.choice([-1, 1], size=u.size) * scale).astype(np.int32)
        h = (rng.integers(-5, 6, size=n) * max(1, scale // 15)).astype(np.int32)
        g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
        jobs.append(psa.Job(ctx, g, 30, T, 9, i0=_schedule(scale > 1, 30)))
        edges.append((n, u, v, j, h))
    psa.jobs_step_batch(ctx, jobs, 13)
    listed = jobs + [jobs[3]]
    hE, hC = psa.jobs_energy_cut(ctx, listed)
    dE = [torch.zeros(j.trials, dtype=torch.int64, device="cuda") for j in listed]
    dC = [torch.zeros(j.trials, dtype=torch.int64, device="cuda") for j in listed]
    psa.jobs_energy_cut(ctx, listed, dE, dC)
    ctx.synchronize()
    for idx, job in enumerate(listed):
        E, C = job.energy_cut()
        np.testing.assert_array_equal(hE[idx], E, err_msg=f"job {idx}")
        np.testing.assert_array_equal(hC[idx], C, err_msg=f"job {idx}")
        np.testing.assert_array_equal(dE[idx].cpu().numpy(), E, err_msg=f"job {idx}")
        np.testing.assert_array_equal(dC[idx].cpu().numpy(), C, err_msg=f"job {idx}")
    for idx, job in enumerate(jobs):
        n, u, v, j, h = edges[idx]
        oE, oC = oracle.energy_cut(n, u, v, j, h, job.read_spins())
        np.testing.assert_array_equal(hE[idx], oE, err_msg=f"job {idx}")
        np.testing.assert_array_equal(hC[idx], oC, err_msg=f"job {idx}")
    assert psa.jobs_energy_cut(ctx, []) == ([], [])
    other = psa.Context(0)
    n, u, v, w = inputs.torus(6, 7, 63)
    g2 = psa.Graph.from_edges(other, n, u, v, w, maxcut=True)
    j2 = psa.Job(other, g2, 10, 4, 1)
    with pytest.raises(psa.PsaError):
        psa.jobs_energy_cut(ctx, [jobs[0], j2])
    j2.close()
    g2.close()
    other.close()
