"""GPU tests of the autotuner: every configuration it can pick gives the
results of the plain run (launch shape and path never change results), the
tuning cache is keyed by shape class, and the measured choice follows the
structure of the graph where the gap is large (rows of ~600 entries ->
matrix cores, short sparse rows -> CSR)."""
import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


@pytest.fixture()
def ctx(psa):
    c = psa.Context(0)
    yield c
    c.close()


KW = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)


def test_autotune_alone_and_tuned_job_exact(psa, ctx):
    n, u, v, w = inputs.gnm(900, 2700, 61)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    r = psa.autotune(ctx, g, 60, 40, 3, probe_steps=6, **KW)
    assert r["candidates"] >= 4            # CSR x4 shapes + dense (+-1 weights)
    assert r["path"] in (psa.PSA_PATH_CSR, psa.PSA_PATH_DENSE)
    assert r["us_per_step"] > 0 and r["csr_us_per_step"] > 0 and r["dense_us_per_step"] > 0
    assert r["us_per_step"] == min(r["csr_us_per_step"], r["dense_us_per_step"])
    assert psa.tune_cache_size(ctx) == 1
    tuned = psa.Job(ctx, g, 60, 40, 3, tune=True, **KW)
    assert psa.tune_cache_size(ctx) == 1   # same class: served from the cache
    plain = psa.Job(ctx, g, 60, 40, 3, path=psa.PSA_PATH_CSR, **KW)
    tuned.step(60)
    plain.step(60)
    np.testing.assert_array_equal(tuned.read_spins(), plain.read_spins())
    lam, dl, thr = oracle.variability(n, 3, 0.1, 0.1, 0.1, 0.8)
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, 60)
    ref = oracle.anneal(n, u, v, -w, None, i0, lam, dl, thr, 3, 0, 2)
    np.testing.assert_array_equal(tuned.read_spins()[:2], ref[0])
    # a job of the same class but another graph is served from the cache too
    n2, u2, v2, w2 = inputs.gnm(905, 2715, 62)
    g2 = psa.Graph.from_edges(ctx, n2, u2, v2, w2, maxcut=True)
    psa.Job(ctx, g2, 60, 40, 3, tune=True, **KW).close()
    assert psa.tune_cache_size(ctx) == 1
    psa.tune_clear(ctx)
    assert psa.tune_cache_size(ctx) == 0


def test_autotune_batch_follows_row_length(psa, ctx):
    n, u, v, w = inputs.erdos_renyi(2000, 0.3, 63)           # ~600 entries a row
    dense_g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    r = psa.autotune(ctx, dense_g, 200, 64, 1, probe_steps=8, batch=True)
    assert r["path"] == psa.PSA_PATH_DENSE, r
    n, u, v, w = inputs.torus(40, 50, 64)                    # 4 entries a row
    sparse_g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    r = psa.autotune(ctx, sparse_g, 200, 64, 1, probe_steps=8, batch=True)
    assert r["path"] == psa.PSA_PATH_CSR, r
    assert psa.tune_cache_size(ctx) == 2


def test_batch_tuning_classes_trials_by_half_octave(psa, ctx):
    """In batched mode the cache keys trial counts by half octave (40 and 44
    share a class, 64 does not); alone, by the exact count."""
    psa.tune_clear(ctx)
    n, u, v, w = inputs.gnm(1000, 3000, 69)
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    psa.tune_get(ctx, g, 50, 40, 1, batch=True)
    psa.tune_get(ctx, g, 50, 44, 1, batch=True)
    assert psa.tune_cache_size(ctx) == 1
    psa.tune_get(ctx, g, 50, 64, 1, batch=True)
    assert psa.tune_cache_size(ctx) == 2
    psa.tune_get(ctx, g, 50, 40, 1)
    psa.tune_get(ctx, g, 50, 44, 1)
    assert psa.tune_cache_size(ctx) == 4
    psa.tune_clear(ctx)


def test_tuned_batch_equals_untuned(psa, ctx):
    specs = [(inputs.erdos_renyi(1200, 0.1, 65), 64, 40),
             (inputs.gnm(1500, 4500, 66), 64, 35),
             (inputs.erdos_renyi(600, 0.3, 67, weights="pm1"), 20, 30),
             (inputs.torus(20, 30, 68), 9, 25)]
    graphs, items, tuned_items = [], [], []
    for (n, u, v, w), T, S in specs:
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        graphs.append(g)
        items.append((g, S, T, 7, dict(KW)))
        tuned_items.append((g, S, T, 7, dict(KW, tune=True)))
    plain = psa.anneal_batch(ctx, items, spins=True)
    tuned = psa.anneal_batch(ctx, tuned_items, spins=True)
    assert psa.tune_cache_size(ctx) >= 1
    for (pS, pE, pC), (tS, tE, tC) in zip(plain, tuned):
        np.testing.assert_array_equal(tS, pS)
        np.testing.assert_array_equal(tE, pE)
        np.testing.assert_array_equal(tC, pC)
