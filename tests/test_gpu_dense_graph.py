"""GPU tests of the dense path's launch modes.  With captured graphs a
quantum of k dense steps is captured once as a HIP graph and replayed for
every later quantum of the same shape: every replay -- with other work
launched eagerly and the host synchronising between replays -- must leave
the spins the oracle computes for that many steps.  The same run launched
step by step, and as one persistent launch per quantum, must match it bit
for bit."""
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


def _run(psa, how, enc):
    """Spins after each quantum of a dense run, with eager CSR work between
    the quanta; also the timing counters of the dense family."""
    ctx = psa.Context(0)
    try:
        ctx.set_dense_launch(how)
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
    (n, u, v, j, h, i0), snaps, tm = _run(psa, psa.PSA_DENSE_LAUNCH_GRAPH, enc)
    assert tm["dense_launches"] == QUANTUM * QUANTA
    assert tm["dense_graph_launches"] == QUANTUM * QUANTA   # one capture, then replays
    lam, dl, thr = oracle.variability(n, SEED, 0.1, 0.1, 0.1, 0.8)
    for q, got in enumerate(snaps):
        ref = oracle.anneal(n, u, v, j, h, i0[:QUANTUM * (q + 1)], lam, dl, thr, SEED, 0, 2)
        np.testing.assert_array_equal(got, ref[0], err_msg=f"after quantum {q}")
    _, eager, tm_off = _run(psa, psa.PSA_DENSE_LAUNCH_STEPS, enc)
    assert tm_off["dense_graph_launches"] == 0 and tm_off["dense_launches"] == QUANTUM * QUANTA
    _, pers, tm_p = _run(psa, psa.PSA_DENSE_LAUNCH_PERSISTENT, enc)
    assert tm_p["dense_graph_launches"] == 0 and tm_p["dense_launches"] == QUANTA  # one launch a quantum
    for q in range(QUANTA):
        np.testing.assert_array_equal(snaps[q], eager[q])
        np.testing.assert_array_equal(snaps[q], pers[q])


def test_persistent_wait_failure_is_reported(psa):
    """A persistent dense quantum whose dependency waits give up (the wait
    bound forced to zero from the host: every kernel still exits normally)
    makes the next dense quantum fail with PSA_EHIP; with the bound restored
    the context runs a fresh job exactly."""
    ctx = psa.Context(0)
    try:
        ctx.set_dense_launch(psa.PSA_DENSE_LAUNCH_PERSISTENT)
        n, u, v, w = inputs.erdos_renyi(600, 0.2, 80)
        g = psa.Graph.from_edges(ctx, n, u, v, -w, maxcut=False)
        i0 = oracle.schedule(12, 0.01, 0.4)
        job = psa.Job(ctx, g, 12, 20, 9, i0=i0, path=psa.PSA_PATH_DENSE, **KW)
        ctx.debug_dense_wait_limit(0)
        job.step(6)
        with pytest.raises(psa.PsaError) as err:
            job.step(6)
        assert err.value.status == psa.PSA_EHIP
        ctx.debug_dense_wait_limit(1 << 20)
        fresh = psa.Job(ctx, g, 12, 20, 9, i0=i0, path=psa.PSA_PATH_DENSE, **KW)
        fresh.step(12)
        lam, dl, thr = oracle.variability(n, 9, 0.1, 0.1, 0.1, 0.8)
        ref = oracle.anneal(n, u, v, -w, None, i0, lam, dl, thr, 9, 0, 2)
        np.testing.assert_array_equal(fresh.read_spins()[:2], ref[0])
        fresh.close()
        job.close()
        g.close()
    finally:
        ctx.close()
