"""GPU tests of the solution-quality harness: its traces, sweeps and cycle
series are the same anneals the library runs directly, aggregated."""
import json

import numpy as np
import pytest

from paper_2601_14476_amd import experiments, inputs

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


@pytest.fixture(scope="module")
def graph(psa, ctx):
    n, u, v, w = inputs.gnm(300, 900, 77)
    return psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)


def test_energy_trace_ends_at_the_anneal(psa, ctx, graph):
    kw = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
    for alg in experiments.ALGORITHMS:
        e = experiments.energy_trace(psa, ctx, graph, 20, 8, 3, alg, **kw)
        assert e.shape == (20, 8)
        _, E, _ = psa.anneal(ctx, graph, 20, 8, 3, spins=False,
                             algorithm=experiments._alg(psa, alg), **kw)
        np.testing.assert_array_equal(e[-1], E)


def test_sweep_and_cycles_aggregate_anneals(psa, ctx, graph):
    rows = experiments.sigma_sweep(psa, ctx, graph, "nu", [0.0, 0.2], 30, 6, 1)
    assert [r["sigma"] for r in rows] == [0.0, 0.2]
    cut0 = psa.anneal(ctx, graph, 30, 6, 1, spins=False)[2]
    assert rows[0]["mean_cut"] == pytest.approx(cut0.mean()) and rows[0]["best_cut"] == cut0.max()
    cut1 = psa.anneal(ctx, graph, 30, 6, 1, spins=False, sigma_nu=0.2, p_mean=0.8)[2]
    assert rows[1]["mean_cut"] == pytest.approx(cut1.mean())
    per = experiments.sigma_sweep(psa, ctx, graph, "nu", [0.3], 12, 4, 1, t_res=10)
    cutp = psa.anneal(ctx, graph, 12, 4, 1, spins=False, sigma_nu=0.3, t_res=10)[2]
    assert per[0]["mean_cut"] == pytest.approx(cutp.mean())
    rows = experiments.cut_vs_cycles(psa, ctx, graph, [5, 40], 6, 2)
    for r in rows:
        cut = psa.anneal(ctx, graph, r["cycles"], 6, 2, spins=False)[2]
        assert r["mean_cut"] == pytest.approx(cut.mean())


def test_command_line(capsys):
    assert experiments.main(["sweep", "--graph", "n2000", "--trials", "4", "--cycles", "20",
                             "--values", "0,0.1", "--factor", "lambda"]) == 0
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["experiment"] == "sweep" and len(out["rows"]) == 2 and out["n"] == 2000
