"""Solution-quality experiments on synthetic stand-ins for the paper's graphs.

The paper reports annealing quality as the mean cut over 100 trials (Methods)
and studies it along three axes, all reproduced here on seeded graphs of the
shapes of Table 1 (G-set itself is not available):

  trace   the energy of every trial after each cycle (as in the energy-versus-
          cycle plots of pSA, TApSA and SpSA, Results);
  sweep   the mean and best cut as one variability factor (sigma_lambda,
          sigma_delta or sigma_nu, Eq. 7) is varied with the others at zero
          (the sensitivity study on G1, Results);
  cycles  the mean cut as the number of annealing cycles grows (the cut-
          versus-time plots on G1 and G81, Results).

Every anneal runs on the GPU through the library (psa.py); this module only
chooses inputs and aggregates results.  Command line:

    python -m paper_2601_14476_amd.experiments trace  --graph g1 --cycles 100
    python -m paper_2601_14476_amd.experiments sweep  --graph g1 --factor nu
    python -m paper_2601_14476_amd.experiments cycles --graph g81

Each prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs

# Table 1 shapes: G1 (G(800, 0.06), +1 weights) and G81 (100 x 200 torus, +-1)
GRAPHS = {
    "g1": ("er", 800, 0.06, 1, "one"),
    "g81": ("torus", 100, 200, 3, "pm1"),
    "n2000": ("gnm", 2000, 6000, 2, "pm1"),
}

ALGORITHMS = ("psa", "spsa", "tapsa")


def _graph(psa, ctx, name):
    n, u, v, w = inputs.make_graph(GRAPHS[name])
    return psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True), n, u.size


def _alg(psa, name):
    return {"psa": psa.PSA_ALG_PSA, "spsa": psa.PSA_ALG_SPSA, "tapsa": psa.PSA_ALG_TAPSA}[name]


def energy_trace(psa, ctx, graph, cycles, trials, seed=0, algorithm="psa", **kw):
    """Energies [cycles][trials] after each cycle (one job stepped a cycle
    at a time; energy and cut on the device)."""
    job = psa.Job(ctx, graph, cycles, trials, seed, algorithm=_alg(psa, algorithm), **kw)
    out = np.zeros((cycles, trials), np.int64)
    for t in range(cycles):
        job.step(1)
        out[t] = job.energy_cut()[0]
    job.close()
    return out


def anneal_cuts(psa, ctx, graph, cycles, trials, seed=0, algorithm="psa", **kw):
    """Final cuts of one anneal of `trials` trials."""
    _, _, cut = psa.anneal(ctx, graph, cycles, trials, seed, spins=False,
                           algorithm=_alg(psa, algorithm), **kw)
    return cut


def sigma_sweep(psa, ctx, graph, factor, values, cycles, trials, seed=0, algorithm="psa",
                t_res=0, p_mean=0.8):
    """Mean, best and spread of the final cut as one variability factor
    takes each of `values` (the others zero).  Timing (factor 'nu') is an
    update probability clip(N(p_mean, sigma^2), 0, 1) (t_res = 0; sigma 0 is
    plain pSA with p = 1) or integer periods of t_res sub-steps."""
    rows = []
    for s in values:
        kw = dict(sigma_lambda=0.0, sigma_delta=0.0, sigma_nu=0.0, p_mean=1.0, t_res=t_res)
        if factor == "lambda":
            kw["sigma_lambda"] = s
        elif factor == "delta":
            kw["sigma_delta"] = s
        elif factor == "nu":
            kw["sigma_nu"] = s
            if t_res == 0 and s > 0:
                kw["p_mean"] = p_mean
        else:
            raise ValueError(f"unknown factor {factor!r}")
        cut = anneal_cuts(psa, ctx, graph, cycles, trials, seed, algorithm, **kw)
        rows.append(dict(sigma=float(s), mean_cut=float(cut.mean()), best_cut=int(cut.max()),
                         std_cut=float(cut.std())))
    return rows


def cut_vs_cycles(psa, ctx, graph, cycle_counts, trials, seed=0, algorithm="psa", **kw):
    """Mean and best final cut for each annealing length."""
    rows = []
    for c in cycle_counts:
        cut = anneal_cuts(psa, ctx, graph, int(c), trials, seed, algorithm, **kw)
        rows.append(dict(cycles=int(c), mean_cut=float(cut.mean()), best_cut=int(cut.max())))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="solution-quality experiments (GPU)")
    ap.add_argument("what", choices=["trace", "sweep", "cycles"])
    ap.add_argument("--graph", default="g1", choices=sorted(GRAPHS))
    ap.add_argument("--algorithm", default="psa", choices=ALGORITHMS)
    ap.add_argument("--trials", type=int, default=100)
    ap.add_argument("--cycles", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--factor", default="nu", choices=["lambda", "delta", "nu"])
    ap.add_argument("--values", default="0,0.05,0.1,0.2,0.5,1.0")
    ap.add_argument("--t-res", type=int, default=0,
                    help="timing as integer periods of this many sub-steps per cycle")
    ap.add_argument("--sigma", type=float, default=0.0, help="trace: sigma of all three factors")
    ap.add_argument("--cycle-counts", default="10,30,100,300,1000")
    args = ap.parse_args(argv)

    from . import psa
    ctx = psa.Context(0)
    graph, n, m = _graph(psa, ctx, args.graph)
    out = dict(experiment=args.what, graph=args.graph, n=n, edges=int(m),
               algorithm=args.algorithm, trials=args.trials, seed=args.seed,
               data="synthetic (seeded stand-in of the Table 1 shape)")
    if args.what == "trace":
        s = args.sigma
        kw = dict(sigma_lambda=s, sigma_delta=s, sigma_nu=s, p_mean=0.8 if s > 0 else 1.0,
                  t_res=args.t_res)
        e = energy_trace(psa, ctx, graph, args.cycles, args.trials, args.seed, args.algorithm, **kw)
        out.update(cycles=args.cycles, sigma=s, t_res=args.t_res,
                   mean_energy=[float(x) for x in e.mean(axis=1)],
                   min_energy=[int(x) for x in e.min(axis=1)])
    elif args.what == "sweep":
        vals = [float(x) for x in args.values.split(",")]
        out.update(cycles=args.cycles, factor=args.factor, t_res=args.t_res,
                   rows=sigma_sweep(psa, ctx, graph, args.factor, vals, args.cycles, args.trials,
                                    args.seed, args.algorithm, t_res=args.t_res))
    else:
        counts = [int(x) for x in args.cycle_counts.split(",")]
        out.update(rows=cut_vs_cycles(psa, ctx, graph, counts, args.trials, args.seed,
                                      args.algorithm, t_res=args.t_res))
    graph.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
