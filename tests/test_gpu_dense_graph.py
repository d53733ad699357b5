"""GPU tests of the dense path's captured step sequences (an opt-in of the
context): a quantum of k dense steps is captured once as a HIP graph and
replayed for every later quantum of the same shape.  Every replay -- with other work launched eagerly
and the host synchronising between replays -- must leave the spins the oracle
computes for that many steps, and the same run with graphs switched off must
match it bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2601_14476_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1, p_mean=0.8)
QUANTUM, QUANTA, TRIALS, SEED = 6, 5, 40, 5


@pytest.fixture(scope="module")
def psa():
    from paper_2601_14476_amd import psa as mod
    return mod


def _run(psa, graphs_on, enc):
    """Spins after each quantum of a dense run, with eager CSR work between
    the quanta; also the timing counters of the dense family."""
    ctx = psa.Context(0)
    try:
        ctx.set_dense_graphs(graphs_on)
        if enc == "t2":
            n, u, v, w = inputs.erdos_renyi(700, 0.2, 77)     # +-1: 2-bit couplings, fp4
            j, h = -w, None
        else:
            rng = np.random.default_rng(78)                  # |J| <= 5: int8 couplings
            n, u, v, w = inputs.erdos_renyi(650, 0.2, 78)
            j = (rng.integers(1, 6, size=w.size) * np.where(rng.random(w.size) < 0.5, -1, 1)).astype(np.int32)
            h = rng.integers(-3, 4, size=n).astype(np.int32)
        g = psa.Graph.from_edges(ctx, n, u, v, j, h=h, maxcut=False)
        steps = QUANTUM * QUANTA
        i0 = oracle.schedule(steps, 0.01, 0.4)
        job = psa.Job(ctx, g, steps, TRIALS, SEED, i0=i0, path=psa.PSA_PATH_DENSE, **KW)
        assert job.info()["path"] == psa.PSA_PATH_DENSE
        on, ou, ov, ow = inputs.gnm(500, 1500, 79)
        og = psa.Graph.from_edges(ctx, on, ou, ov, ow, maxcut=True)
        other = psa.Job(ctx, og, 3 * QUANTA, 8, 3, path=psa.PSA_PATH_CSR, **KW)
        ctx.set_timing(True)
        ctx.timing()
        snaps = []
        for _ in range(QUANTA):
            job.step(QUANTUM)
            other.step(3)
            ctx.synchronize()
            snaps.append(job.read_spins()[:2].copy())
        tm = ctx.timing()
        job.close()
        other.close()
        g.close()
        og.close()
        return (n, u, v, j, h, i0), snaps, tm
    finally:
        ctx.close()


@pytest.mark.parametrize("enc", ["t2", "i8"])
def test_dense_graph_replays_match_oracle_and_eager(psa, enc):
    (n, u, v, j, h, i0), snaps, tm = _run(psa, True, enc)
    assert tm["dense_launches"] == QUANTUM * QUANTA
    assert tm["dense_graph_launches"] == QUANTUM * QUANTA   # one capture, then replays
    lam, dl, thr = oracle.variability(n, SEED, 0.1, 0.1, 0.1, 0.8)
    for q, got in enumerate(snaps):
        ref = oracle.anneal(n, u, v, j, h, i0[:QUANTUM * (q + 1)], lam, dl, thr, SEED, 0, 2)
        np.testing.assert_array_equal(got, ref[0], err_msg=f"after quantum {q}")
    _, eager, tm_off = _run(psa, False, enc)
    assert tm_off["dense_graph_launches"] == 0
    for q in range(QUANTA):
        np.testing.assert_array_equal(snaps[q], eager[q])
