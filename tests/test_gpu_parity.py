"""GPU parity: every result of the HIP path, through the C ABI, equals the
oracle's bit for bit (spins, local fields, energies, cuts).

Small cases are compared element by element over whole trajectories; the
full-size workloads (G1-shaped ER n=800; n=2,000 sparse with variability;
the G81-shaped 100x200 torus with 1,024 trials and 5,000 steps) run in the
launch configuration the benchmark times and are compared on sampled
trials, which the oracle recomputes independently (trials never interact).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu
ONE24 = 1 << 24


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


@pytest.fixture(scope="module")
def ctx(psa):
    c = psa.Context(0)
    yield c
    c.close()


def _graph(psa, ctx, n, u, v, w, h=None):
    return psa.Graph.from_edges(ctx, n, u, v, w, h=h, maxcut=True)


def _oracle_params(n, u, v, w, steps, seed, sl, sd, sn, pm):
    i0, lo, hi = oracle.schedule_paper(n, u, v, -w, steps)
    lam, dlt, thr = oracle.variability(n, seed, sl, sd, sn, pm)
    return i0, lam, dlt, thr


def _job(psa, ctx, g, spec, trials=None, steps=None, block=0, tpw=0, lpt=0):
    return psa.Job(ctx, g, steps or spec["steps"], trials or spec["trials"], spec["seed"],
                   sigma_lambda=spec["sigma_lambda"], sigma_delta=spec["sigma_delta"],
                   sigma_nu=spec["sigma_nu"], p_mean=spec["p_mean"], block=block,
                   trials_per_group=tpw, lanes_per_task=lpt)


# ----------------------------------------------------------------------------
# graph ingestion and schedule endpoints
# ----------------------------------------------------------------------------
def test_graph_info_and_paper_schedule(psa, ctx):
    for name in ("c1", "c2", "c3"):
        spec = inputs.workload(name)
        n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
        g = _graph(psa, ctx, n, u, v, w)
        info = g.info()
        assert info["n"] == n and info["edges"] == u.size and info["nnz"] == 2 * u.size
        assert info["w_total"] == int(w.sum())
        assert info["mean_s"] == oracle.mean_s(n, u, v, -w)
        lo, hi = g.schedule_paper()
        _, olo, ohi = oracle.schedule_paper(n, u, v, -w, 10)
        assert (lo, hi) == (olo, ohi)
        g.close()


def test_invalid_graphs_rejected(psa, ctx):
    z = np.array([0], np.int32)
    o = np.array([1], np.int32)
    with pytest.raises(psa.PsaError) as e:
        psa.Graph.from_edges(ctx, 2, z, z, o)               # self loop
    assert e.value.status == psa.PSA_EINVAL
    with pytest.raises(psa.PsaError):
        psa.Graph.from_edges(ctx, 2, np.array([0, 1], np.int32), np.array([1, 0], np.int32),
                             np.array([1, 1], np.int32))    # repeated pair
    with pytest.raises(psa.PsaError):
        psa.Graph.from_edges(ctx, 2, z, np.array([5], np.int32), o)   # out of range
    with pytest.raises(psa.PsaError):
        psa.Graph.from_edges(ctx, 2, z, o, np.array([1 << 24], np.int32))
    with pytest.raises(psa.PsaError):                         # asymmetric CSR
        psa.Graph.from_csr(ctx, 2, [0, 1, 1], [1], [1])


# ----------------------------------------------------------------------------
# initial spins, local field, energy / cut
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("trials", [1, 3, 4, 10, 101, 1023])
def test_initial_spins(psa, ctx, trials):
    n, u, v, w = inputs.gnm(257, 700, 1)
    g = _graph(psa, ctx, n, u, v, w)
    job = psa.Job(ctx, g, steps=5, trials=trials, seed=12345)
    np.testing.assert_array_equal(job.read_spins(), oracle.init_spins(n, 12345, 0, trials))


def _random_ising(n, m, seed, jmax=5):
    rng = np.random.default_rng(seed)
    _, u, v, _ = inputs.gnm(n, m, seed)
    j = rng.integers(1, jmax + 1, size=u.size) * rng.choice([-1, 1], size=u.size)
    h = rng.integers(-7, 8, size=n)
    return n, u, v, j.astype(np.int32), h.astype(np.int32)


@pytest.mark.parametrize("n,m,trials", [(1, 0, 5), (50, 0, 4), (300, 1500, 9), (2048, 9000, 64)])
def test_local_field_and_energy(psa, ctx, n, m, trials):
    n, u, v, j, h = _random_ising(n, m, 3)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    job = psa.Job(ctx, g, steps=3, trials=trials, seed=1, i0_min=0.1, i0_max=1.0)
    rng = np.random.default_rng(5)
    s = rng.choice([-1, 1], size=(trials, n)).astype(np.int8)
    job.write_spins(s, 0)
    np.testing.assert_array_equal(job.read_spins(), s)
    np.testing.assert_array_equal(job.local_field(), oracle.local_field(n, u, v, j, h, s))
    E, C = job.energy_cut()
    oE, oC = oracle.energy_cut(n, u, v, j, h, s)
    np.testing.assert_array_equal(E, oE)
    np.testing.assert_array_equal(C, oC)


# ----------------------------------------------------------------------------
# trajectories, step by step
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name,trials,steps,tpw,lpt", [
    ("c1", 10, 25, 1, 1), ("c1", 10, 25, 1, 4), ("c1", 10, 25, 4, 0),
    ("c2", 100, 12, 1, 1), ("c2", 100, 12, 1, 2), ("c2", 100, 12, 1, 4), ("c2", 100, 12, 4, 0)])
def test_trajectory_every_step(psa, ctx, name, trials, steps, tpw, lpt):
    spec = inputs.workload(name)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    g = _graph(psa, ctx, n, u, v, w)
    S = spec["steps"]
    job = _job(psa, ctx, g, spec, trials=trials, tpw=tpw, lpt=lpt)
    i0, lam, dlt, thr = _oracle_params(n, u, v, w, S, spec["seed"], spec["sigma_lambda"],
                                       spec["sigma_delta"], spec["sigma_nu"], spec["p_mean"])
    ref = oracle.init_spins(n, spec["seed"], 0, trials)
    np.testing.assert_array_equal(job.read_spins(), ref)
    for t in range(steps):
        job.step(1)
        ref = oracle.run(n, u, v, -w, None, i0, lam, dlt, thr, spec["seed"], 0, trials, t,
                         t + 1, ref)
        got = job.read_spins()
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)
            pytest.fail(f"{name} step {t}: {len(bad)} spins differ, first {bad[:5].tolist()}")
    np.testing.assert_array_equal(job.local_field(), oracle.local_field(n, u, v, -w, None, ref))


def _compare_full(psa, ctx, name, sample, block=0, **over):
    spec = inputs.workload(name, **over)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    T, S = spec["trials"], spec["steps"]
    _say(f"[parity] {name}: n={n} trials={T} steps={S} block={block} sample={sample}")
    g = _graph(psa, ctx, n, u, v, w)
    job = _job(psa, ctx, g, spec, block=block)
    job.step(S)
    E, C = job.energy_cut()
    spins = job.read_spins()
    i0, lam, dlt, thr = _oracle_params(n, u, v, w, S, spec["seed"], spec["sigma_lambda"],
                                       spec["sigma_delta"], spec["sigma_nu"], spec["p_mean"])
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(min(len(sample), 16)) as ex:
        res = list(ex.map(lambda k: oracle.anneal(n, u, v, -w, None, i0, lam, dlt, thr,
                                                  spec["seed"], k, k + 1), sample))
    for k, (os_, oE, oC) in zip(sample, res):
        np.testing.assert_array_equal(spins[k], os_[0], err_msg=f"{name} trial {k} spins")
        assert E[k] == oE[0] and C[k] == oC[0], (name, k, E[k], oE[0], C[k], oC[0])
    # energy / cut of every trial against the oracle's evaluation of GPU spins
    oE_all, oC_all = oracle.energy_cut(n, u, v, -w, None, spins)
    np.testing.assert_array_equal(E, oE_all)
    np.testing.assert_array_equal(C, oC_all)
    return spins, E, C


def test_full_c1_all_trials(psa, ctx):
    _compare_full(psa, ctx, "c1", list(range(10)))


def test_full_c2_sampled_trials(psa, ctx):
    _compare_full(psa, ctx, "c2", [0, 1, 2, 3, 4, 37, 50, 96, 98, 99])


def test_full_c3_sampled_trials(psa, ctx):
    """G81-shaped torus, 1,024 trials, 5,000 steps: trials in the first,
    a middle and the last workgroup."""
    _compare_full(psa, ctx, "c3", [0, 513, 1023])


# ----------------------------------------------------------------------------
# edge cases and invariances
# ----------------------------------------------------------------------------
def test_launch_geometry_does_not_change_results(psa, ctx):
    spec = inputs.workload("c2", steps=60, trials=13)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    g = _graph(psa, ctx, n, u, v, w)
    outs = []
    for block, tpw, lpt in ((256, 1, 1), (512, 4, 0), (1024, 1, 1), (1024, 4, 0), (0, 0, 0),
                            (256, 1, 2), (1024, 1, 2), (512, 1, 4), (1024, 1, 4)):
        job = psa.Job(ctx, g, spec["steps"], spec["trials"], spec["seed"],
                      sigma_lambda=spec["sigma_lambda"], sigma_delta=spec["sigma_delta"],
                      sigma_nu=spec["sigma_nu"], p_mean=spec["p_mean"], block=block,
                      trials_per_group=tpw, lanes_per_task=lpt)
        job.step(spec["steps"])
        outs.append(job.read_spins())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_stepping_composes_and_resumes(psa, ctx):
    spec = inputs.workload("c2", steps=40, trials=8)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    g = _graph(psa, ctx, n, u, v, w)
    a = _job(psa, ctx, g, spec)
    a.step(40)
    b = _job(psa, ctx, g, spec)
    for k in (1, 2, 7, 30):
        b.step(k)
    assert b.position == 40
    np.testing.assert_array_equal(a.read_spins(), b.read_spins())
    # checkpoint at step 17, resume in a fresh job
    c = _job(psa, ctx, g, spec)
    c.step(17)
    ck = c.read_spins()
    d = _job(psa, ctx, g, spec)
    d.write_spins(ck, 17)
    d.step(100)
    assert d.position == 40
    np.testing.assert_array_equal(d.read_spins(), a.read_spins())
    # reset returns to the initial state
    a.reset()
    np.testing.assert_array_equal(a.read_spins(), oracle.init_spins(n, spec["seed"], 0, 8))


def test_degenerate_cases(psa, ctx):
    # single p-bit, no couplings, bias and offset
    e = np.zeros(0, np.int32)
    g = psa.Graph.from_edges(ctx, 1, e, e, e, h=np.array([2], np.int32), maxcut=False)
    i0 = oracle.schedule(7, 0.1, 2.0)
    lam = np.array([1.3], np.float32)
    dl = np.array([-0.4], np.float32)
    thr = np.array([ONE24 // 3], np.uint32)
    job = psa.Job(ctx, g, 7, 6, seed=9, i0=i0, lam=lam, delta=dl, thr24=thr)
    job.step(7)
    ref = oracle.anneal(1, e, e, e, np.array([2], np.int32), i0, lam, dl, thr, 9, 0, 6)
    np.testing.assert_array_equal(job.read_spins(), ref[0])
    # zero update probability: spins frozen
    n, u, v, w = inputs.gnm(40, 90, 2)
    g2 = _graph(psa, ctx, n, u, v, w)
    job2 = psa.Job(ctx, g2, 20, 5, seed=4, p_mean=0.0)
    s0 = job2.read_spins()
    job2.step(20)
    np.testing.assert_array_equal(job2.read_spins(), s0)
    # one step, explicit schedule, integer weights > 1 and biases
    n, u, v, j, h = _random_ising(70, 200, 8)
    g3 = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    i0 = np.array([0.37], np.float32)
    lam, dl, thr = oracle.variability(n, 3, 0.2, 0.3, 0.2, 0.7)
    job3 = psa.Job(ctx, g3, 1, 7, seed=3, i0=i0, sigma_lambda=0.2, sigma_delta=0.3,
                   sigma_nu=0.2, p_mean=0.7)
    job3.step(1)
    ref3 = oracle.anneal(n, u, v, j, h, i0, lam, dl, thr, 3, 0, 7)
    np.testing.assert_array_equal(job3.read_spins(), ref3[0])
    E, C = job3.energy_cut()
    np.testing.assert_array_equal(E, ref3[1])
    np.testing.assert_array_equal(C, ref3[2])


def test_anneal_one_call_matches_job(psa, ctx):
    spec = inputs.workload("c1", steps=50, trials=6)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    g = _graph(psa, ctx, n, u, v, w)
    S, E, C = psa.anneal(ctx, g, 50, 6, 0)
    job = _job(psa, ctx, g, spec)
    job.step(50)
    np.testing.assert_array_equal(S, job.read_spins())
    E2, C2 = job.energy_cut()
    np.testing.assert_array_equal(E, E2)
    np.testing.assert_array_equal(C, C2)


def test_device_outputs(psa, ctx):
    import torch
    spec = inputs.workload("c1", steps=30, trials=10)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    dctx = psa.Context(0, stream)
    g = _graph(psa, dctx, n, u, v, w)
    job = _job(psa, dctx, g, spec)
    job.step(30)
    s = torch.empty((10, n), dtype=torch.int8, device="cuda")
    E = torch.empty(10, dtype=torch.int64, device="cuda")
    C = torch.empty(10, dtype=torch.int64, device="cuda")
    job.read_spins(s)
    job.energy_cut(E, C)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s.cpu().numpy(), job.read_spins())
    hE, hC = job.energy_cut()
    np.testing.assert_array_equal(E.cpu().numpy(), hE)
    np.testing.assert_array_equal(C.cpu().numpy(), hC)
    job.close()
    g.close()
    dctx.close()
    torch.cuda.set_stream(torch.cuda.default_stream())


def _star_plus_ring(n, hub_degree, seed):
    """A hub joined to `hub_degree` p-bits plus a ring: one row longer than 255."""
    rng = np.random.default_rng(seed)
    u = [0] * hub_degree
    v = list(range(1, hub_degree + 1))
    for i in range(1, n):
        u.append(i)
        v.append(i % (n - 1) + 1)
    u, v = np.array(u, np.int32), np.array(v, np.int32)
    key = np.minimum(u, v).astype(np.int64) * n + np.maximum(u, v)
    _, first = np.unique(key, return_index=True)
    keep = np.sort(first)
    u, v = u[keep], v[keep]
    keep = u != v
    u, v = u[keep], v[keep]
    w = rng.choice([-1, 1], size=u.size).astype(np.int32)
    return n, u, v, w


@pytest.mark.parametrize("kind", ["unit", "int", "big", "hub", "wide"])
@pytest.mark.parametrize("tpw,lpt", [(1, 1), (1, 2), (1, 4), (4, 0)])
def test_edge_encodings_match_oracle(psa, ctx, kind, tpw, lpt):
    """Every edge encoding of the anneal kernel (0/1-byte mirror, SWAR words,
    packed 32-bit, separate col/val), with the edges in LDS and (kind "wide":
    200 KB of edges, rows of ~50) in global memory, against the oracle, 30
    steps."""
    if kind == "unit":
        n, u, v, w = inputs.gnm(603, 2500, 11)
        j, h = -w, None
    elif kind == "wide":
        n, u, v, w = inputs.gnm(2000, 50000, 15)
        j, h = -w, None
    elif kind == "int":
        n, u, v, j, h = _random_ising(603, 2500, 12)
    elif kind == "big":                       # |J| >= 2^15: col/val pairs
        n, u, v, j, h = _random_ising(211, 700, 13, jmax=3)
        j = (j * 20000).astype(np.int32)
        h = (h * 1000).astype(np.int32)
    else:                                     # a row of degree 300 (> 255)
        n, u, v, w = _star_plus_ring(500, 300, 14)
        j, h = -w, None
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    T, S = 9, 30
    lam, dl, thr = oracle.variability(n, 21, 0.2, 0.3, 0.2, 0.7)
    i0 = oracle.schedule(S, 0.02, 0.5) if kind != "big" else oracle.schedule(S, 1e-5, 1e-4)
    job = psa.Job(ctx, g, S, T, seed=21, i0=i0, sigma_lambda=0.2, sigma_delta=0.3,
                  sigma_nu=0.2, p_mean=0.7, trials_per_group=tpw, lanes_per_task=lpt)
    job.step(S)
    ref = oracle.anneal(n, u, v, j, h, i0, lam, dl, thr, 21, 0, T)
    np.testing.assert_array_equal(job.read_spins(), ref[0])
    E, C = job.energy_cut()
    np.testing.assert_array_equal(E, ref[1])
    np.testing.assert_array_equal(C, ref[2])


@pytest.mark.parametrize("n,trials,kind", [(1, 3, "unit"), (63, 7, "int"), (64, 16, "unit"),
                                           (65, 33, "int"), (300, 64, "unit"), (1000, 100, "int"),
                                           (257, 1, "unit"), (129, 5, "scaled"), (700, 40, "one"),
                                           (1300, 130, "one"), (385, 64, "scaled"), (520, 70, "ferro"),
                                           (333, 64, "zeros")])
def test_dense_path_matches_oracle(psa, ctx, n, trials, kind):
    """Dense matrix-core path against the oracle and against the CSR path:
    identical spins, energies and cuts.  "one" (+1 weights: every J = -1) and
    "ferro" (every J = +2) take the 1-bit encoding, "unit" (+-1) and "scaled"
    (+-3) the 2-bit one, "int" (|J| <= 5) and "zeros" (+-1 with some stored
    zero couplings) the int8 one; sizes span several 256-row groups, coupling
    chunks and trial tiles with ragged tails."""
    if kind in ("unit", "one", "scaled", "ferro", "zeros"):
        if n > 1:
            p = 0.3 if kind not in ("one", "ferro") else 0.08
            _, u, v, w = inputs.erdos_renyi(n, p, 40 + n, weights="one" if kind in ("one", "ferro") else "pm1")
        else:
            u = v = w = np.zeros(0, np.int32)
        if kind == "scaled":
            w = 3 * w
        if kind == "ferro":
            w = -2 * w
        if kind == "zeros":
            w = w.copy()
            w[::7] = 0
        j, h = -w, None
    else:
        n, u, v, j, h = _random_ising(n, 4 * n, 41 + n, jmax=5)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    S = 20
    i0 = oracle.schedule(S, 0.01, 0.4)
    kw = dict(i0=i0, sigma_lambda=0.1, sigma_delta=0.2, sigma_nu=0.1, p_mean=0.8)
    dense = psa.Job(ctx, g, S, trials, 7, path=psa.PSA_PATH_DENSE, **kw)
    expect = {"one": 3, "ferro": 3, "unit": 2, "scaled": 2, "int": 1, "zeros": 1}[kind]
    assert dense.info()["dense_encoding"] == expect
    csr = psa.Job(ctx, g, S, trials, 7, path=psa.PSA_PATH_CSR, **kw)
    dense.step(7)
    dense.step(13)
    csr.step(S)
    np.testing.assert_array_equal(dense.read_spins(), csr.read_spins())
    lam, dl, thr = oracle.variability(n, 7, 0.1, 0.2, 0.1, 0.8)
    k = min(trials, 3)
    ref = oracle.anneal(n, u, v, j, h, i0, lam, dl, thr, 7, 0, k)
    np.testing.assert_array_equal(dense.read_spins()[:k], ref[0])
    E, C = dense.energy_cut()
    np.testing.assert_array_equal(E[:k], ref[1])
    np.testing.assert_array_equal(C[:k], ref[2])


def test_dense_path_rejects_wide_couplings(psa, ctx):
    """Couplings of several magnitudes, one above int8, have no dense encoding
    (a single magnitude, however large, takes the 2-bit or 1-bit one)."""
    g = psa.Graph.from_edges(ctx, 3, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                             np.array([300, 1], np.int32), maxcut=False)
    with pytest.raises(psa.PsaError) as e:
        psa.Job(ctx, g, 5, 2, 0, i0_min=0.001, i0_max=0.01, path=psa.PSA_PATH_DENSE)
    assert e.value.status == psa.PSA_EUNSUPPORTED


def test_objects_outlive_their_creators_handles(psa):
    """The context and graph stay alive while a job needs them: dropping the
    creator's handles first must neither crash nor change results."""
    n, u, v, w = inputs.gnm(300, 900, 3)
    c = psa.Context(0)
    g = psa.Graph.from_edges(c, n, u, v, w)
    job = psa.Job(c, g, 20, 5, 1)
    ref = psa.Job(c, g, 20, 5, 1)
    ref.step(20)
    expect = ref.read_spins()
    ref.close()
    g.close()
    c.close()                 # job still holds both
    job.step(20)
    np.testing.assert_array_equal(job.read_spins(), expect)
    job.close()


@pytest.mark.parametrize("kind,tpw,lpt,path", [
    ("unit", 1, 1, "csr"), ("unit", 1, 2, "csr"), ("unit", 1, 4, "csr"), ("unit", 4, 0, "csr"),
    ("int", 1, 2, "csr"), ("int", 4, 0, "csr"), ("unit", 0, 0, "dense"), ("int", 0, 0, "dense"),
    ("long", 1, 4, "csr")])
def test_spsa_trajectories_match_oracle(psa, ctx, kind, tpw, lpt, path):
    """Stalled p-bits (Eq. 5): spins after every chunk of steps equal the
    oracle's on every path and launch shape (held inputs carried between
    launches on the device)."""
    if kind == "unit":
        n, u, v, w = inputs.gnm(333, 1400, 91)
        j, h = -w, None
    elif kind == "long":  # rows of ~90 edges: one-row lanes past their cached slots
        n, u, v, w = inputs.erdos_renyi(300, 0.3, 91, weights="pm1")
        j, h = -w, None
    else:
        n, u, v, j, h = _random_ising(301, 1300, 92, jmax=4)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    S, T = 24, 11
    i0 = oracle.schedule(S, 0.02, 0.9)
    sig = (0.1, 0.2, 0.1, 0.8)
    lam, dl, thr = oracle.variability(n, 13, *sig)
    job = psa.Job(ctx, g, S, T, seed=13, i0=i0, sigma_lambda=sig[0], sigma_delta=sig[1],
                  sigma_nu=sig[2], p_mean=sig[3], trials_per_group=tpw, lanes_per_task=lpt,
                  path=psa.PSA_PATH_DENSE if path == "dense" else psa.PSA_PATH_CSR,
                  algorithm=psa.PSA_ALG_SPSA, p_stall=0.5)
    ref = oracle.init_spins(n, 13, 0, T)
    x = None
    t = 0
    for k in (1, 6, 9, 8):
        job.step(k)
        ref, x = oracle.run_spsa(n, u, v, j, h, i0, lam, dl, thr, 1 << 23, 13, 0, T, t, t + k,
                                 ref, x)
        t += k
        np.testing.assert_array_equal(job.read_spins(), ref, err_msg=f"after step {t}")
    E, C = job.energy_cut()
    rE, rC = oracle.energy_cut(n, u, v, j, h, ref)
    np.testing.assert_array_equal(E, rE)
    np.testing.assert_array_equal(C, rC)


def test_spsa_edge_cases(psa, ctx):
    """p_stall 0 is pSA; p_stall 1 freezes every input at step 0 (matches the
    oracle); a reset re-forms the inputs; resuming an SpSA job mid-run from
    spins alone is refused."""
    n, u, v, w = inputs.gnm(200, 700, 93)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    kw = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
    a = psa.anneal(ctx, g, 30, 7, 4, **kw)
    b = psa.anneal(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_SPSA, p_stall=0.0, **kw)
    np.testing.assert_array_equal(a[0], b[0])
    job = psa.Job(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_SPSA, p_stall=1.0, **kw)
    job.step(30)
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, 30)
    lam, dl, thr = oracle.variability(n, 4, 0.1, 0.1, 0.1, 0.8)
    ref = oracle.anneal_spsa(n, u, v, -w, None, i0, lam, dl, thr, 1 << 24, 4, 0, 7)
    np.testing.assert_array_equal(job.read_spins(), ref[0])
    job.reset()
    job.step(30)
    np.testing.assert_array_equal(job.read_spins(), ref[0])
    with pytest.raises(psa.PsaError) as e:
        job.write_spins(job.read_spins(), 5)
    assert e.value.status == psa.PSA_EUNSUPPORTED
    with pytest.raises(psa.PsaError):
        psa.Job(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_SPSA, p_stall=1.5)


@pytest.mark.parametrize("kind,tpw,lpt,path,window", [
    ("unit", 1, 1, "csr", 4), ("unit", 1, 2, "csr", 4), ("unit", 1, 4, "csr", 3),
    ("unit", 4, 0, "csr", 4), ("int", 1, 2, "csr", 4), ("int", 4, 0, "csr", 2),
    ("unit", 0, 0, "dense", 4), ("int", 0, 0, "dense", 3), ("long", 1, 4, "csr", 4)])
def test_tapsa_trajectories_match_oracle(psa, ctx, kind, tpw, lpt, path, window):
    """Time-averaged p-bits (Eq. 4): spins after every chunk of steps equal
    the oracle's on every path and launch shape (field windows carried
    between launches on the device, start-up averages included)."""
    if kind == "unit":
        n, u, v, w = inputs.gnm(333, 1400, 94)
        j, h = -w, None
    elif kind == "long":  # rows of ~90 edges: one-row lanes past their cached slots
        n, u, v, w = inputs.erdos_renyi(300, 0.3, 94, weights="pm1")
        j, h = -w, None
    else:
        n, u, v, j, h = _random_ising(301, 1300, 95, jmax=4)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    S, T = 24, 11
    i0 = oracle.schedule(S, 0.02, 0.9)
    sig = (0.1, 0.2, 0.1, 0.8)
    lam, dl, thr = oracle.variability(n, 17, *sig)
    job = psa.Job(ctx, g, S, T, seed=17, i0=i0, sigma_lambda=sig[0], sigma_delta=sig[1],
                  sigma_nu=sig[2], p_mean=sig[3], trials_per_group=tpw, lanes_per_task=lpt,
                  path=psa.PSA_PATH_DENSE if path == "dense" else psa.PSA_PATH_CSR,
                  algorithm=psa.PSA_ALG_TAPSA, window=window)
    ref = oracle.init_spins(n, 17, 0, T)
    ring = None
    t = 0
    for k in (1, 2, 6, 7, 8):
        job.step(k)
        ref, ring = oracle.run_tapsa(n, u, v, j, h, i0, lam, dl, thr, window, 17, 0, T, t,
                                     t + k, ref, ring)
        t += k
        np.testing.assert_array_equal(job.read_spins(), ref, err_msg=f"after step {t}")
    E, C = job.energy_cut()
    rE, rC = oracle.energy_cut(n, u, v, j, h, ref)
    np.testing.assert_array_equal(E, rE)
    np.testing.assert_array_equal(C, rC)


def test_tapsa_edge_cases(psa, ctx):
    """A window of one is pSA; resuming a TApSA job mid-run from spins alone
    is refused; windows outside [1, 64] are rejected."""
    n, u, v, w = inputs.gnm(200, 700, 96)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    kw = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
    a = psa.anneal(ctx, g, 30, 7, 4, **kw)
    b = psa.anneal(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_TAPSA, window=1, **kw)
    np.testing.assert_array_equal(a[0], b[0])
    job = psa.Job(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_TAPSA, window=4, **kw)
    job.step(10)
    with pytest.raises(psa.PsaError) as e:
        job.write_spins(job.read_spins(), 5)
    assert e.value.status == psa.PSA_EUNSUPPORTED
    for bad in (0, 65):
        with pytest.raises(psa.PsaError):
            psa.Job(ctx, g, 30, 7, 4, algorithm=psa.PSA_ALG_TAPSA, window=bad)


@pytest.mark.parametrize("kind,tpw,lpt,path,t_res", [
    ("unit", 1, 2, "csr", 10), ("unit", 1, 4, "csr", 10), ("unit", 1, 1, "csr", 7),
    ("unit", 4, 0, "csr", 10), ("int", 1, 2, "csr", 10), ("int", 4, 0, "csr", 3),
    ("unit", 0, 0, "dense", 10), ("int", 0, 0, "dense", 5), ("long", 1, 4, "csr", 10)])
def test_period_mode_matches_oracle(psa, ctx, kind, tpw, lpt, path, t_res):
    """Period-mode timing (the listing's count mod nu gate at t_res sub-steps
    per cycle): spins after every chunk of cycles equal the oracle's on every
    path and launch shape."""
    if kind == "unit":
        n, u, v, w = inputs.gnm(333, 1400, 97)
        j, h = -w, None
    elif kind == "long":  # rows of ~90 edges: one-row lanes past their cached slots
        n, u, v, w = inputs.erdos_renyi(300, 0.3, 97, weights="pm1")
        j, h = -w, None
    else:
        n, u, v, j, h = _random_ising(301, 1300, 98, jmax=4)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    S, T = 12, 11
    i0 = oracle.schedule(S, 0.02, 0.9)
    lam, dl, _ = oracle.variability(n, 19, 0.1, 0.2, 0.3, 1.0)
    per = oracle.periods(n, 19, 0.3, t_res)
    job = psa.Job(ctx, g, S, T, seed=19, i0=i0, sigma_lambda=0.1, sigma_delta=0.2, sigma_nu=0.3,
                  trials_per_group=tpw, lanes_per_task=lpt, t_res=t_res,
                  path=psa.PSA_PATH_DENSE if path == "dense" else psa.PSA_PATH_CSR)
    ref = oracle.init_spins(n, 19, 0, T)
    t = 0
    for k in (1, 4, 7):
        job.step(k)
        ref = oracle.run_period(n, u, v, j, h, i0, lam, dl, per, t_res, 19, 0, T, t, t + k, ref)
        t += k
        np.testing.assert_array_equal(job.read_spins(), ref, err_msg=f"after cycle {t}")
    E, C = job.energy_cut()
    rE, rC = oracle.energy_cut(n, u, v, j, h, ref)
    np.testing.assert_array_equal(E, rE)
    np.testing.assert_array_equal(C, rC)


def _resident_k(n, block):
    """p-bits per lane of the resident period sweep (0: records sweep)."""
    b = block or 1024
    if n > 2048:
        return 0
    for k in {1024: (1, 2), 512: (1, 2, 4), 256: (1, 2, 4, 8)}[b]:
        if k * b >= n:
            return k
    return 0


@pytest.mark.parametrize("block", [0, 256, 512])
@pytest.mark.parametrize("case", ["classes64", "classes65", "period_one", "pair_edges",
                                  "rows_in_memory", "n3100", "n5000", "sparse_firing",
                                  "long_rows", "int_weights", "n2048"])
def test_period_class_sweep_matches_oracle(psa, ctx, case, block):
    """The period-mode sweep over period classes (one trial per workgroup):
    resident lanes (1, 2, 4 or 8 p-bits per lane at 256, 512 or 1,024 lanes;
    graphs of up to 2,048 p-bits with 16-bit edge words) or the records
    sweep (larger graphs, couplings too large for the packed edge words, too
    many p-bits for the block's lanes).  Spins after chunks of cycles equal
    the oracle's for up to 64 distinct periods (more fall back to the full
    sweep), a class of period 1 (fires at every sub-step), rows in device
    memory, periods so long that most sub-steps fire nothing, rows longer
    than the cached edges, integer couplings with biases, and n = 2,048."""
    t_res, S, T, seed = 10, 12, 7, 23
    h = None
    if case == "pair_edges":
        n, u, v, j, h = _random_ising(400, 1500, 31, jmax=4)
        j[::7] *= 9000       # |J| up to 36,000: no 16-bit coupling field
    elif case == "rows_in_memory":
        n, u, v, w = inputs.erdos_renyi(1500, 0.4, 32, weights="pm1")
        j = -w
    elif case == "n3100":
        n, u, v, w = inputs.gnm(3100, 9000, 33)
        j = -w
    elif case == "n5000":
        n, u, v, w = inputs.gnm(5000, 15000, 38)
        j = -w
    elif case == "long_rows":  # degrees ~20-60: past 12 and 16 cached edges
        n, u, v, w = inputs.gnm(1800, 36000, 35)
        j = -w
    elif case == "int_weights":  # couplings up to 4 and biases: packed words
        n, u, v, j, h = _random_ising(600, 2400, 36, jmax=4)
    elif case == "n2048":  # the largest graph on resident lanes
        n, u, v, w = inputs.gnm(2048, 7000, 37)
        j = -w
    else:
        n, u, v, w = inputs.gnm(700, 2500, 34)
        j = -w
    idx = np.arange(n)
    per = {"classes64": idx % 64 + 1, "classes65": idx % 65 + 1, "period_one": idx % 3 + 1,
           "sparse_firing": 29 + 8 * (idx % 3)}.get(case)
    if per is None:
        per = oracle.periods(n, seed, 0.3, t_res)
    per = np.ascontiguousarray(per, dtype=np.uint32)
    g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
    i0 = oracle.schedule(S, 0.02, 0.9)
    lam, dl, _ = oracle.variability(n, seed, 0.1, 0.2, 0.0, 1.0)
    job = psa.Job(ctx, g, S, T, seed=seed, i0=i0, sigma_lambda=0.1, sigma_delta=0.2,
                  t_res=t_res, period=per, trials_per_group=1, path=psa.PSA_PATH_CSR, block=block)
    classes = len(np.unique(per))
    info = job.info()
    assert info["period_classes"] == (classes if classes <= 64 else 0)
    k = _resident_k(n, block) if classes <= 64 and case != "pair_edges" else 0
    assert info["period_resident"] == k
    ref = oracle.init_spins(n, seed, 0, T)
    t = 0
    for k in (1, 4, 7):
        job.step(k)
        ref = oracle.run_period(n, u, v, j, h, i0, lam, dl, per, t_res, seed, 0, T, t, t + k, ref)
        t += k
        np.testing.assert_array_equal(job.read_spins(), ref, err_msg=f"{case} after cycle {t}")
    E, C = job.energy_cut()
    rE, rC = oracle.energy_cut(n, u, v, j, h, ref)
    np.testing.assert_array_equal(E, rE)
    np.testing.assert_array_equal(C, rC)


def test_period_mode_edge_cases(psa, ctx):
    """t_res 1 with no timing spread is pSA; explicit periods are used as
    given; period mode with SpSA, zero periods and too many sub-steps are
    refused; a period-mode job resumes from its spins (no other state)."""
    n, u, v, w = inputs.gnm(200, 700, 99)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    a = psa.anneal(ctx, g, 30, 7, 4, sigma_lambda=0.1, sigma_delta=0.1)
    b = psa.anneal(ctx, g, 30, 7, 4, sigma_lambda=0.1, sigma_delta=0.1, t_res=1)
    np.testing.assert_array_equal(a[0], b[0])
    per = np.arange(n, dtype=np.uint32) % 13 + 1
    job = psa.Job(ctx, g, 20, 5, 6, t_res=10, period=per)
    job.step(20)
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, 20)
    lam, dl, _ = oracle.variability(n, 6, 0.0, 0.0, 0.0, 1.0)
    ref = oracle.anneal_period(n, u, v, -w, None, i0, lam, dl, per, 10, 6, 0, 5)
    np.testing.assert_array_equal(job.read_spins(), ref[0])
    mid = psa.Job(ctx, g, 20, 5, 6, t_res=10, period=per)
    mid.step(8)
    resumed = psa.Job(ctx, g, 20, 5, 6, t_res=10, period=per)
    resumed.write_spins(mid.read_spins(), 8)
    resumed.step(12)
    np.testing.assert_array_equal(resumed.read_spins(), ref[0])
    with pytest.raises(psa.PsaError) as e:
        psa.Job(ctx, g, 20, 5, 6, t_res=10, algorithm=psa.PSA_ALG_SPSA)
    assert e.value.status == psa.PSA_EUNSUPPORTED
    with pytest.raises(psa.PsaError):
        psa.Job(ctx, g, 20, 5, 6, t_res=10, period=np.zeros(n, np.uint32))
    with pytest.raises(psa.PsaError):
        psa.Job(ctx, g, 1 << 20, 5, 6, t_res=10)


@pytest.mark.parametrize("n,lpt", [(2048, 2), (2049, 0), (1024, 4), (1025, 4)])
def test_fast_layout_boundaries(psa, ctx, n, lpt):
    """Sizes at the edge of the one-trial fast layout (every task a lane pair
    or quad of its own, at most 1,024 lanes): n = 2,048 with two lanes per
    task is the largest that takes it; n = 2,049 falls back to one lane per
    task with cached edge indices; n = 1,025 with four lanes per task cannot
    hold every task and walks slots.  Each against the oracle, 25 steps."""
    m = 3 * n
    nn, u, v, w = inputs.gnm(n, m, 120 + n)
    g = psa.Graph.from_edges(ctx, nn, u, v, w, maxcut=True)
    S, T = 25, 5
    i0 = oracle.schedule(S, 0.02, 0.9)
    lam, dl, thr = oracle.variability(nn, 31, 0.1, 0.2, 0.2, 0.7)
    job = psa.Job(ctx, g, S, T, seed=31, i0=i0, sigma_lambda=0.1, sigma_delta=0.2,
                  sigma_nu=0.2, p_mean=0.7, trials_per_group=1, lanes_per_task=lpt,
                  path=psa.PSA_PATH_CSR)
    job.step(11)
    job.step(S - 11)
    ref = oracle.anneal(nn, u, v, -w, None, i0, lam, dl, thr, 31, 0, T)
    np.testing.assert_array_equal(job.read_spins(), ref[0])


@pytest.mark.parametrize("p", [0.12, 0.3])
def test_one_row_lanes_past_cached_slots(psa, ctx, p):
    """Four lanes per task (one row per lane) on the fast layout cache 64 slot
    addresses per lane; G(400, p) rows of about 48 (p = 0.12) and 120 edges
    (p = 0.3) end before and after the cached slots, and wavefronts mix both
    near 64.  Against the oracle, 20 steps."""
    nn, u, v, w = inputs.erdos_renyi(400, p, 71, weights="pm1")
    g = psa.Graph.from_edges(ctx, nn, u, v, w, maxcut=True)
    deg = np.bincount(np.concatenate([u, v]), minlength=nn)
    S, T = 20, 4
    i0 = oracle.schedule(S, 0.02, 0.9)
    lam, dl, thr = oracle.variability(nn, 19, 0.1, 0.2, 0.2, 0.7)
    job = psa.Job(ctx, g, S, T, seed=19, i0=i0, sigma_lambda=0.1, sigma_delta=0.2,
                  sigma_nu=0.2, p_mean=0.7, trials_per_group=1, lanes_per_task=4,
                  path=psa.PSA_PATH_CSR)
    _say(f"n=400 p={p} degree {deg.min()}..{deg.max()}")
    job.step(7)
    job.step(S - 7)
    ref = oracle.anneal(nn, u, v, -w, None, i0, lam, dl, thr, 19, 0, T)
    np.testing.assert_array_equal(job.read_spins(), ref[0])


@pytest.mark.parametrize("window", [4, 40])
def test_tapsa_windows_in_lds_and_device_memory(psa, ctx, window):
    """TApSA on the fast layout: a window of 4 on n = 1,500 keeps the windows
    in LDS (24 KB), 40 keeps them in device memory (240 KB); both resume
    across launches and equal the oracle."""
    n, u, v, w = inputs.gnm(1500, 4500, 97)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    S, T = 30, 6
    i0 = oracle.schedule(S, 0.02, 0.9)
    lam, dl, thr = oracle.variability(n, 23, 0.1, 0.1, 0.1, 0.8)
    job = psa.Job(ctx, g, S, T, seed=23, i0=i0, sigma_lambda=0.1, sigma_delta=0.1,
                  sigma_nu=0.1, p_mean=0.8, trials_per_group=1, lanes_per_task=2,
                  path=psa.PSA_PATH_CSR, algorithm=psa.PSA_ALG_TAPSA, window=window)
    ref = oracle.init_spins(n, 23, 0, T)
    ring = None
    t = 0
    for k in (3, 9, 18):
        job.step(k)
        ref, ring = oracle.run_tapsa(n, u, v, -w, None, i0, lam, dl, thr, window, 23, 0, T,
                                     t, t + k, ref, ring)
        t += k
        np.testing.assert_array_equal(job.read_spins(), ref, err_msg=f"after step {t}")


def test_four_trial_state_beyond_lds_falls_back(psa, ctx):
    """With 1,024 trials the planner takes four trials per workgroup, whose
    spin state (2 x 4 bytes per p-bit) does not fit LDS at n = 21,000; it
    then runs one trial per workgroup instead.  Sampled trials against the
    oracle."""
    n, u, v, w = inputs.gnm(21000, 42000, 131)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    S, T = 6, 1024
    job = psa.Job(ctx, g, S, T, 5, sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8,
                  path=psa.PSA_PATH_CSR)
    assert job.info()["trials_per_group"] == 1
    job.step(S)
    spins = job.read_spins()
    i0, lam, dl, thr = _oracle_params(n, u, v, w, S, 5, 0.1, 0.1, 0.1, 0.8)
    for k in (0, 511, 1023):
        ref = oracle.anneal(n, u, v, -w, None, i0, lam, dl, thr, 5, k, k + 1)
        np.testing.assert_array_equal(spins[k], ref[0][0], err_msg=f"trial {k}")
