"""Seeded synthetic inputs shaped like the paper's MAX-CUT workloads.

This module only generates inputs (graphs, job mixes, arrival times); it
holds none of the annealing arithmetic, so both the GPU path and the
oracle can be fed from it.

The paper evaluates on G-set graphs (Table 1): random graphs with +1
weights (G1: 800 nodes, 19,176 edges) and toroidal grids with +-1 weights
(G81: 20,000 nodes, 40,000 edges).  Those files are not part of this
project; the generators below produce graphs of the same shapes instead:

* ``erdos_renyi(800, 0.06)`` has an expected C(800,2)*0.06 = 19,176 edges,
  G1's count;
* ``torus(100, 200)`` has exactly 40,000 edges, G81's count and structure.

Every generator returns ``(n, u, v, w)``: the node count and int32 arrays of
the undirected edges (each pair once, no self loops) and their MAX-CUT
weights.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "erdos_renyi", "gnm", "torus", "workload", "WORKLOADS", "batch_jobs",
    "serve_trace",
]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _weights(rng, m, weights):
    if weights == "one":
        return np.ones(m, np.int32)
    if weights == "pm1":
        return np.where(rng.random(m) < 0.5, 1, -1).astype(np.int32)
    raise ValueError(f"unknown weights {weights!r}")


def erdos_renyi(n, p, seed, weights="one"):
    """G(n, p): every pair i < j is an edge independently with probability p."""
    rng = _rng(seed)
    us, vs = [], []
    for i in range(n - 1):
        hit = np.nonzero(rng.random(n - 1 - i) < p)[0]
        us.append(np.full(hit.size, i, np.int32))
        vs.append((hit + i + 1).astype(np.int32))
    u = np.concatenate(us) if us else np.zeros(0, np.int32)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int32)
    return n, u, v, _weights(rng, u.size, weights)


def gnm(n, m, seed, weights="pm1"):
    """G(n, m): m distinct pairs drawn uniformly without replacement."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges for a simple graph")
    rng = _rng(seed)
    keys = np.zeros(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        ok = a != b
        lo = np.minimum(a, b)[ok].astype(np.int64)
        hi = np.maximum(a, b)[ok].astype(np.int64)
        cand = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(cand, return_index=True)
        keys = cand[np.sort(first)]
    keys = keys[:m]
    u = (keys // n).astype(np.int32)
    v = (keys % n).astype(np.int32)
    return n, u, v, _weights(rng, m, weights)


def torus(rows, cols, seed, weights="pm1"):
    """2-D toroidal grid: (r, c) joined to (r, c+1) and (r+1, c), indices mod."""
    if rows < 3 or cols < 3:
        raise ValueError("torus sides must be >= 3 for a simple graph")
    rng = _rng(seed)
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    node = (r * cols + c).ravel()
    right = (r * cols + (c + 1) % cols).ravel()
    down = (((r + 1) % rows) * cols + c).ravel()
    u = np.concatenate([node, node]).astype(np.int32)
    v = np.concatenate([right, down]).astype(np.int32)
    return rows * cols, u, v, _weights(rng, u.size, weights)


# Workloads.  `seed` keys the annealing randomness (Philox key); the graph
# seed is separate.  sigma_* are the standard deviations of Eq. 7; p_mean
# is the mean per-step update probability of the timing factor.
WORKLOADS = {
    # Plain pSA on a G1-shaped random graph, weights +1, 1,000 steps, 10 trials.
    "c1": dict(graph=("er", 800, 0.06, 1, "one"), steps=1000, trials=10,
               seed=0, sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0,
               p_mean=1.0),
    # Random sparse graph n=2,000, mean degree 6, +-1; variability 0.1.
    "c2": dict(graph=("gnm", 2000, 6000, 2, "pm1"), steps=2000, trials=100,
               seed=0, sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1,
               p_mean=0.8),
    # G81-shaped 100x200 torus, +-1, variability 0.1, 5,000 steps, 1,024 trials.
    "c3": dict(graph=("torus", 100, 200, 3, "pm1"), steps=5000, trials=1024,
               seed=0, sigma_lambda=0.1, sigma_delta=0.1, sigma_nu=0.1,
               p_mean=0.8),
}


def make_graph(spec):
    kind = spec[0]
    if kind == "er":
        _, n, p, gseed, wts = spec
        return erdos_renyi(n, p, gseed, wts)
    if kind == "gnm":
        _, n, m, gseed, wts = spec
        return gnm(n, m, gseed, wts)
    if kind == "torus":
        _, r, c, gseed, wts = spec
        return torus(r, c, gseed, wts)
    raise ValueError(f"unknown graph kind {kind!r}")


def workload(name, **override):
    """Return a dict with the graph arrays and run parameters of a workload."""
    spec = dict(WORKLOADS[name])
    spec.update(override)
    n, u, v, w = make_graph(spec["graph"])
    spec.update(name=name, n=n, u=u, v=v, w=w)
    return spec


def batch_jobs(count=256, seed=4, trials=64, steps=1000):
    """A mix of uneven graphs for the batched launch.

    Half are G(n, p) with p ~ U[0.02, 0.1] and weights +1 (dense enough for
    the matrix-core path), half G(n, n*d/2) with d ~ U{4..8} and +-1
    weights; n ~ U{800..5000}.  Job g uses graph seed 1000*seed + g and
    annealing seed g.
    """
    rng = _rng(seed)
    jobs = []
    for g in range(count):
        n = int(rng.integers(800, 5001))
        gseed = 1000 * seed + g
        if g % 2 == 0:
            p = float(rng.uniform(0.02, 0.1))
            gspec = ("er", n, p, gseed, "one")
        else:
            d = int(rng.integers(4, 9))
            gspec = ("gnm", n, n * d // 2, gseed, "pm1")
        jobs.append(dict(graph=gspec, steps=steps, trials=trials, seed=g,
                         sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0,
                         p_mean=1.0))
    return jobs


def serve_trace(rate=50.0, duration=120.0, seed=5, n_range=(800, 20000),
                deg_range=(4, 50), steps_range=(1000, 10000),
                trials_range=(32, 256), sigmas=(0.0, 0.05, 0.1, 0.2)):
    """Poisson arrivals and the job each one carries.

    Returns a list of (arrival_time_s, job_spec) sorted by time; job id j
    uses graph seed 100000 + j and annealing seed j.
    """
    rng = _rng(seed)
    t = 0.0
    out = []
    j = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.integers(deg_range[0], deg_range[1] + 1))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        trials = int(rng.integers(trials_range[0], trials_range[1] + 1))
        sigma = float(sigmas[int(rng.integers(0, len(sigmas)))])
        m = min(n * d // 2, n * (n - 1) // 2)
        spec = dict(graph=("gnm", n, m, 100000 + j, "pm1"), steps=steps,
                    trials=trials, seed=j, sigma_lambda=sigma,
                    sigma_delta=sigma, sigma_nu=sigma,
                    p_mean=0.8 if sigma > 0 else 1.0)
        out.append((t, spec))
        j += 1
    return out
