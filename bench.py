#!/usr/bin/env python3
"""Throughput of the pSA hot path on one MI355X.

One benchmark step = one whole anneal of the workload with its inputs
already resident in HBM: reset the spins of every trial (initial-state
kernel), run all sweeps (the persistent anneal kernel), and reduce energy
and cut per trial into device buffers.  The metric is p-bit updates per
second, n * trials * steps per anneal / wall time of the timed steps.

Default workload: the G81-shaped 100 x 200 torus (n=20,000, 40,000 edges,
+-1 weights), timing/intensity/offset variability sigma 0.1 (update
probability mean 0.8), 5,000 sweeps, 1,024 trials -- the largest single-GPU
configuration.  Other workloads: --workload c1 (G1-shaped ER, n=800, 1,000
sweeps, 10 trials), c2 (random sparse n=2,000, 6,000 edges, 2,000 sweeps,
100 trials), c4 (batched mix of 256 graphs), c4-dense (the dense step alone)
and c5 (serving trace).

Besides the contract fields the JSON line carries:
  roofline     -- the anneal kernel's algorithmic VALU lane-operations per
                  launch over its average duration (HIP events on the
                  library's stream) against the chip's VALU issue rate, with
                  three operation counts side by side: the gfx950 lower bound
                  (the headline fraction), the workload table's estimate, and
                  the lane-instructions the kernel issued (rocprofv3 counters
                  under profiles/, while the sources are unchanged);
  cpu_baseline -- the oracle timed on this host's cores on a bounded sample
                  of the same workload (trials spread over threads).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic 32-bit lane-operations per p-bit update: the fewest VALU
# instructions the method's arithmetic takes on gfx950 (a lower bound on what
# a kernel issues).  One Philox4x32-10 block = 10 rounds x (2 32x32->64
# multiplies, one instruction each, + 2 three-input XOR) = 40, shared by the
# 4 p-bits of a task; the timing gate needs a second block.
PHILOX_BLOCK_OPS = 40
OPS_R_MAP = 4          # shift-or, subtract, convert, scale
OPS_GATE_MAP = 2       # shift, compare
OPS_PREACT = 3.25      # int->float, + delta, * a  (a = I0*lambda once per quad)
OPS_DECIDE = 11        # tanh estimate (clamp, scale, 2^v, +1, reciprocal, fma,
                       # sign), distance to r, two compares, select
# neighbour term per edge: a three-input add takes two neighbour bytes of one
# trial; one add of a packed word takes a neighbour of four trials
OPS_EDGE_ONE_TRIAL = 0.5
OPS_EDGE_FOUR_TRIALS = 0.25

# MI355X: 256 CUs x 4 SIMD x 16 lanes, one 32-bit VALU op per lane per clock
# at 2.4 GHz (the 157.3 TFLOP/s FP32 figure counts an FMA as 2 and dual issue).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
OPS_STALL = 3  # shift-compare of the stall word, select of the held input
OPS_WINDOW = 2  # window sum: add the entering field, subtract the leaving one
OPS_MEAN = 10  # window mean: convert, correctly rounded divide
OPS_PERIOD = 6  # period test: convert, reciprocal, multiply, truncate, multiply-subtract, compare
MFMA_I8_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak, TOP/s
MFMA_F4_PEAK_TOPS = 10100.0  # dense fp4 matrix-core peak, TFLOP/s
DENSE_LAUNCH = {"steps": 0, "graph": 1, "persistent": 2}
HBM_PEAK_GBS = 8000.0

# The workload table's own estimate of the VALU work per update (written
# before any kernel, for a generic 32-bit ISA): about 100 lane-operations per
# Philox4x32-10 block, of which an update takes a quarter (r) or a half (r and
# the timing gate), about 20 FP32 operations for the pre-activation and tanh,
# and one add per neighbour.  gfx950 forms each 32x32->64 product in one
# instruction and each three-way XOR in another, so a block takes 40, which is
# why the lower bound above is the headline count.
PLAN_PHILOX_BLOCK_OPS = 100
PLAN_FP32_OPS = 20

# Host threads the oracle may use: the CPU share of one GPU on the GPU hosts
# (16), whatever the machine's core count.
CPU_SHARE_THREADS = 16

TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "hbm_traffic_by_workload.md")
ISSUE_TABLE = os.path.join(ROOT, "profiles", "valu_issue_by_workload.md")


# The sources each measured kernel is compiled from: its own file, the
# per-update arithmetic and the argument structures it reads (and, for the
# dense step, the host file that cuts its launch into work items).
KERNEL_SOURCES = {
    "anneal_kernel": ["anneal.hip", "device_math.hpp", "engine.hpp"],
    "dense_step_kernel": ["dense.hip", "device_math.hpp", "engine.hpp", "batch.cpp"],
    "period_kernel": ["period.hip", "device_math.hpp", "engine.hpp"],
}


def source_digest(kernel: str) -> str:
    """sha256 (first 16 hex digits) over the sources `kernel` is compiled
    from (names and bytes, in the listed order): the counter tables under
    profiles/ are keyed on it, so a row stops applying once the kernel's
    code changes, and only then."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_14476_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload`, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE table under profiles/ (already scaled by the
    copy-kernel calibration), or None when no row matches or the library's
    sources differ from those the counters were taken on."""
    try:
        with open(TRAFFIC_TABLE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = source_digest(kernel)
    for ln in lines:
        cells = [c.strip().strip("`") for c in ln.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0] == workload and cells[1] == kernel and cells[5] == digest:
            return int(cells[4].replace(",", ""))
    return None


def measured_issue(workload: str, kernel: str):
    """(issued VALU lane-instructions per update, VALU busy fraction) of
    `kernel` on `workload` from the rocprofv3 SQ_INSTS_VALU table under
    profiles/, or None when no row matches the library's current sources."""
    try:
        with open(ISSUE_TABLE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = source_digest(kernel)
    for ln in lines:
        cells = [c.strip().strip("`") for c in ln.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == workload and cells[1] == kernel and cells[6] == digest:
            return float(cells[4]), float(cells[5])
    return None


def plan_ops_per_update(degree: float, timing: bool) -> float:
    """The workload table's estimate of VALU lane-operations per update."""
    return PLAN_PHILOX_BLOCK_OPS * (0.5 if timing else 0.25) + PLAN_FP32_OPS + degree


def host_cpu():
    """(logical cores of this host, CPU model name)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def ops_per_update(field_ops: float, timing: bool, algorithm: str = "psa") -> float:
    """Algorithmic 32-bit lane-operations of one p-bit update; field_ops is
    the neighbour term (mean degree x the per-edge cost of the sweep).  SpSA
    adds a quarter Philox block for the stall word and its compare and
    select; TApSA the window-sum update and the mean (convert, divide)."""
    spsa = algorithm == "spsa"
    philox = PHILOX_BLOCK_OPS / 4 * ((2 if timing else 1) + (1 if spsa else 0))
    extra = OPS_STALL if spsa else (OPS_WINDOW + OPS_MEAN if algorithm == "tapsa" else 0)
    return (philox + OPS_R_MAP + (OPS_GATE_MAP if timing else 0) + field_ops
            + OPS_PREACT + OPS_DECIDE + extra)


def edge_ops(job_info) -> float:
    """Per-edge cost of the neighbour term for the sweep a job runs."""
    return OPS_EDGE_FOUR_TRIALS if job_info["trials_per_group"] == 4 else OPS_EDGE_ONE_TRIAL


def cpu_baseline(spec, budget_s: float = 15.0, stall24=None, window=None, t_res=None):
    """Time the oracle on a bounded sample: the first `k` trials over the
    full schedule, k chosen so the single-thread work is about budget_s.
    stall24 / window: time the SpSA / TApSA oracle instead."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    S = spec["steps"]
    i0, _, _ = oracle.schedule_paper(n, u, v, -w, S)
    lam, dlt, thr = oracle.variability(n, spec["seed"], spec["sigma_lambda"],
                                       spec["sigma_delta"], spec["sigma_nu"],
                                       spec["p_mean"])
    # calibrate: one trial, a few steps
    cal_steps = max(1, min(S, 50))
    t0 = time.perf_counter()
    per = oracle.periods(n, spec["seed"], spec["sigma_nu"], t_res) if t_res else None
    if t_res:
        oracle.run_period(n, u, v, -w, None, i0, lam, dlt, per, t_res, spec["seed"], 0, 1, 0,
                          cal_steps, oracle.init_spins(n, spec["seed"], 0, 1))
    elif window is not None:
        oracle.run_tapsa(n, u, v, -w, None, i0, lam, dlt, thr, window, spec["seed"], 0, 1, 0,
                         cal_steps, oracle.init_spins(n, spec["seed"], 0, 1))
    elif stall24 is None:
        oracle.run(n, u, v, -w, None, i0, lam, dlt, thr, spec["seed"], 0, 1, 0, cal_steps,
                   oracle.init_spins(n, spec["seed"], 0, 1))
    else:
        oracle.run_spsa(n, u, v, -w, None, i0, lam, dlt, thr, stall24, spec["seed"], 0, 1, 0,
                        cal_steps, oracle.init_spins(n, spec["seed"], 0, 1))
    per_update = (time.perf_counter() - t0) / (n * cal_steps)
    host_cores, model = host_cpu()
    cores = min(host_cores, CPU_SHARE_THREADS)
    trials = max(1, min(spec["trials"], int(budget_s / (per_update * n * S))))
    trials = max(min(cores, spec["trials"]), trials)
    bounds = np.linspace(0, trials, min(cores, trials) + 1).astype(int)
    parts = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(parts)) as ex:
        if t_res:
            list(ex.map(lambda ab: oracle.anneal_period(n, u, v, -w, None, i0, lam, dlt, per,
                                                        t_res, spec["seed"], ab[0], ab[1]),
                        parts))
        elif window is not None:
            list(ex.map(lambda ab: oracle.anneal_tapsa(n, u, v, -w, None, i0, lam, dlt, thr,
                                                       window, spec["seed"], ab[0], ab[1]),
                        parts))
        elif stall24 is None:
            list(ex.map(lambda ab: oracle.anneal(n, u, v, -w, None, i0, lam, dlt, thr,
                                                 spec["seed"], ab[0], ab[1]), parts))
        else:
            list(ex.map(lambda ab: oracle.anneal_spsa(n, u, v, -w, None, i0, lam, dlt, thr,
                                                      stall24, spec["seed"], ab[0], ab[1]),
                        parts))
    dt = time.perf_counter() - t0
    updates = n * trials * S
    return {"value": updates / dt, "unit": "p-bit updates/s", "cores": len(parts),
            "kind": "oracle",
            "sample": f"{trials} of {spec['trials']} trials x all {S} steps x n={n} "
                      f"({updates:.3g} updates, {dt:.2f} s wall on {len(parts)} threads)",
            "host_cores": host_cores, "cpu_model": model,
            "single_thread_updates_per_s": 1.0 / per_update}


def cpu_baseline_batch(graphs, steps, trials, budget_s: float = 15.0):
    """Time the oracle on a bounded sample of the batched mix: the first
    trials of the first graphs (alternately G(n, p) and degree 4-8) over the
    full schedule, about budget_s of single-thread work, spread over up to 16
    threads.  graphs: [(n, u, v, w, seed)]."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    host_cores, model = host_cpu()
    cores = min(host_cores, CPU_SHARE_THREADS)
    units = []   # (graph index, trial)
    prepared = []
    est = 0.0
    for gi, (n, u, v, w, seed) in enumerate(graphs):
        i0, _, _ = oracle.schedule_paper(n, u, v, -w, steps)
        lam, dlt, thr = oracle.variability(n, seed, 0.0, 0.0, 0.0, 1.0)
        prepared.append((n, u, v, w, seed, i0, lam, dlt, thr))
        # calibrate on this graph: one trial, a few steps
        cal = min(steps, 20)
        t0 = time.perf_counter()
        oracle.run(n, u, v, -w, None, i0, lam, dlt, thr, seed, 0, 1, 0, cal,
                   oracle.init_spins(n, seed, 0, 1))
        per_trial = (time.perf_counter() - t0) / cal * steps
        k = 0
        while k < min(trials, 4) and est < budget_s:
            units.append((gi, k))
            est += per_trial
            k += 1
        if est >= budget_s:
            break

    def run(unit):
        gi, k = unit
        n, u, v, w, seed, i0, lam, dlt, thr = prepared[gi]
        oracle.anneal(n, u, v, -w, None, i0, lam, dlt, thr, seed, k, k + 1)
        return n * steps

    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(cores, len(units))) as ex:
        updates = sum(ex.map(run, units))
    dt = time.perf_counter() - t0
    used = sorted({gi for gi, _ in units})
    return {"value": updates / dt, "unit": "p-bit updates/s", "cores": min(cores, len(units)),
            "kind": "oracle",
            "sample": f"{len(units)} trials of graphs {used[0]}..{used[-1]} of the mix x all "
                      f"{steps} steps ({updates:.3g} updates, {dt:.2f} s wall)",
            "host_cores": host_cores, "cpu_model": model}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c4-dense", "c5"])
    ap.add_argument("--rate", type=float, default=50.0, help="c5: arrivals per second")
    ap.add_argument("--duration", type=float, default=20.0, help="c5: seconds of arrivals")
    ap.add_argument("--quantum", type=int, default=250, help="c5: steps per scheduling quantum")
    ap.add_argument("--max-resident", type=int, default=128, help="c5: resident job slots")
    ap.add_argument("--alone-sample", type=int, default=12,
                    help="c5: served jobs rerun one at a time for the comparison")
    ap.add_argument("--graphs", type=int, default=256,
                    help="c4: graphs in the batch (256 = the workload; fewer for profiling)")
    ap.add_argument("--no-tune", action="store_true",
                    help="c5: cost-model path choice instead of the autotuner")
    ap.add_argument("--algorithm", default="psa", choices=["psa", "spsa", "tapsa"],
                    help="c1-c3: update rule (pSA, Eq. 3; stalled p-bits, Eq. 5; "
                         "time-averaged p-bits, Eq. 4)")
    ap.add_argument("--p-stall", type=float, default=0.5, help="SpSA stall probability")
    ap.add_argument("--window", type=int, default=4, help="TApSA window (alpha)")
    ap.add_argument("--t-res", type=int, default=0,
                    help="c1-c3: period-mode timing with this many sub-steps per cycle "
                         "(0 = update-probability timing)")
    ap.add_argument("--path", default="auto", choices=["auto", "csr", "dense"],
                    help="c1-c3: field path")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tpw", type=int, default=0, help="trials per workgroup (0 = auto)")
    ap.add_argument("--lpt", type=int, default=0, help="lanes per 4-p-bit task (0 = auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense-launch", choices=["steps", "persistent", "graph"], default="steps",
                    help="c4, c4-dense, c5: how a dense quantum is launched (one launch per step, "
                         "one persistent launch, or per-step launches replayed from a captured "
                         "graph)")
    ap.add_argument("--dense-weights", choices=["one", "pm1"], default="one",
                    help="c4-dense: +1 weights (1-bit couplings, the workload) or +-1 weights "
                         "(2-bit couplings)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times); "
                         "used to scale the HBM traffic counters")
    ap.add_argument("--source-digest", action="store_true",
                    help="only print the digest of the library's sources that the HBM "
                         "traffic table is keyed on")
    args = ap.parse_args()
    if args.source_digest:
        for k in KERNEL_SOURCES:
            print(k, source_digest(k))
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark measures one GPU only (asked for --gpus {args.gpus}); "
              "trials and jobs shard across GPUs without communication, but no "
              "multi-GPU figure is produced here.", file=sys.stderr)
        sys.exit(2)

    pool = None
    if args.workload == "c5":
        # the serving benchmark's graph producers, started before anything
        # in this process touches the GPU
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(processes=8)
    import torch
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy, "copies": 3}), flush=True)
        return
    from paper_2601_14476_amd import inputs, psa

    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c4-dense":
        return bench_dense(args)
    if args.workload == "c5":
        return bench_serve(args, pool)
    spec = inputs.workload(args.workload)
    n, u, v, w = spec["n"], spec["u"], spec["v"], spec["w"]
    T, S = spec["trials"], spec["steps"]
    torch.cuda.set_device(0)
    # A non-default torch stream: the library launches on it and the HIP
    # events below are recorded on it, so they bracket the kernels exactly.
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = psa.Context(0, stream)
    ctx.set_dense_launch(DENSE_LAUNCH[args.dense_launch])
    g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
    info = g.info()
    spsa = args.algorithm == "spsa"
    alg = {"psa": psa.PSA_ALG_PSA, "spsa": psa.PSA_ALG_SPSA, "tapsa": psa.PSA_ALG_TAPSA}[args.algorithm]
    job = psa.Job(ctx, g, S, T, spec["seed"], sigma_lambda=spec["sigma_lambda"],
                  sigma_delta=spec["sigma_delta"], sigma_nu=spec["sigma_nu"],
                  p_mean=spec["p_mean"], block=args.block, trials_per_group=args.tpw,
                  lanes_per_task=args.lpt, path={"auto": psa.PSA_PATH_AUTO, "csr": psa.PSA_PATH_CSR,
                                                 "dense": psa.PSA_PATH_DENSE}[args.path],
                  algorithm=alg, p_stall=args.p_stall, window=args.window, t_res=args.t_res)
    E = torch.empty(T, dtype=torch.int64, device="cuda")
    C = torch.empty(T, dtype=torch.int64, device="cuda")

    def one_step(ev=None):
        job.reset()
        if ev is not None:
            ev[0].record(stream)
        job.step(S)
        if ev is not None:
            ev[1].record(stream)
        job.energy_cut(E, C)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    updates = n * T * S
    value = updates * args.steps / wall
    timing = spec["sigma_nu"] > 0 or spec["p_mean"] < 1.0
    jinfo = job.info()
    field_ops = 0.0 if jinfo["path"] == psa.PSA_PATH_DENSE else info["nnz"] / n * edge_ops(jinfo)
    opu = ops_per_update(field_ops, timing, args.algorithm)
    if args.t_res > 0:
        # period mode: per cycle and p-bit, the expected number of firings
        # (t_res / period), each an ungated update that draws a whole Philox
        # block (the other three words of its counter belong to p-bits that
        # fire at other sub-steps); the sweep over period classes tests
        # periods per class, not per p-bit
        per = psa.periods_draw(n, spec["seed"], spec["sigma_nu"], args.t_res)
        fires = float(np.mean(args.t_res / per.astype(np.float64)))
        opu = fires * (ops_per_update(field_ops, False) + PHILOX_BLOCK_OPS * 3 / 4)
        if jinfo["period_classes"] == 0:
            opu += args.t_res * OPS_PERIOD
    achieved = opu * updates / (kernel_ms * 1e-3) / 1e12
    kname = ("dense_step_kernel" if job.dense else
             "period_kernel" if args.t_res > 0 and jinfo["period_classes"] > 0 else "anneal_kernel")
    default_launch = (args.algorithm == "psa" and not args.t_res and args.path == "auto"
                      and not (args.block or args.tpw or args.lpt))
    # the three operation counts side by side (plain pSA in probability mode)
    op_counts = {"gfx950_lower_bound": opu}
    if args.algorithm == "psa" and not args.t_res and not job.dense:
        op_counts["workload_table_estimate"] = plan_ops_per_update(info["nnz"] / n, timing)
    issue = measured_issue(args.workload, kname) if default_launch else None
    if issue is not None:
        op_counts["issued_measured"] = issue[0]
    fracs = {k: v * updates / (kernel_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS
             for k, v in op_counts.items()}
    line = {
        "metric": "p-bit updates/s (n x trials x steps / s), 1 GPU",
        "value": value,
        "unit": "p-bit updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 spins / int32 field / f32 pre-activation",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "graph": spec["graph"][0],
            "n": n, "edges": int(u.size), "trials": T, "sweeps": S,
            "sigma_lambda": spec["sigma_lambda"], "sigma_delta": spec["sigma_delta"],
            "sigma_nu": spec["sigma_nu"], "p_mean": spec["p_mean"],
            "updates_per_anneal": updates,
            "algorithm": args.algorithm, "p_stall": args.p_stall if spsa else None,
            "window": args.window if args.algorithm == "tapsa" else None,
            "t_res": args.t_res or None,
            "path": "dense" if job.dense else "csr",
        },
        "roofline": {
            "bound": "alu",
            "kernel": kname,
            "achieved": achieved,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS,
            # counters were taken in the default launch of each workload only
            "traffic": measured_traffic(args.workload, kname) if default_launch else None,
            "ops_per_update": opu,
            "op_counts_per_update": op_counts,
            "fracs_by_op_count": fracs,
            "valu_busy_measured": issue[1] if issue is not None else None,
            "kernel_ms": kernel_ms,
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(
            spec, stall24=int(args.p_stall * 2 ** 24) if spsa else None,
            window=args.window if args.algorithm == "tapsa" else None,
            t_res=args.t_res or None)
    print(json.dumps(line), flush=True)
    job.close()
    g.close()
    ctx.close()


def bench_batch(args):
    """256 graphs of uneven size (n in [800, 5000]; half G(n, p) with +1
    weights, p in [0.02, 0.1]; half random degree 4-8 with +-1 weights), 64
    trials, 1,000 sweeps each, all resident.  Path and launch shape of every
    job come from the autotuner (batched mode, per shape class; tuning time
    is reported apart, as set-up).  One batched launch per step sequence
    versus the same anneals one graph at a time (each tuned for running
    alone) on the same stream."""
    import torch
    from paper_2601_14476_amd import inputs, psa
    specs = inputs.batch_jobs(count=args.graphs)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = psa.Context(0, stream)
    ctx.set_dense_launch(DENSE_LAUNCH[args.dense_launch])
    graphs, jobs, alone, outs = [], [], [], []
    updates = 0
    valu_ops = 0.0       # CSR jobs
    dense_valu = 0.0     # dense jobs' epilogue
    dense_bytes = 0.0
    mfma_ops = 0.0
    dense_jobs = 0
    t_tune = 0.0
    for sp in specs:
        n, u, v, w = inputs.make_graph(sp["graph"])
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        info = g.info()
        t0 = time.perf_counter()
        rb = psa.tune_get(ctx, g, sp["steps"], sp["trials"], sp["seed"], batch=True)
        ra = psa.tune_get(ctx, g, sp["steps"], sp["trials"], sp["seed"], batch=False)
        t_tune += time.perf_counter() - t0
        kb = psa.tune_kwargs(rb)
        if kb["trials_per_group"] == 0:
            kb["trials_per_group"] = 1
        jobs.append(psa.Job(ctx, g, sp["steps"], sp["trials"], sp["seed"], **kb))
        alone.append(psa.Job(ctx, g, sp["steps"], sp["trials"], sp["seed"], **psa.tune_kwargs(ra)))
        graphs.append(g)
        outs.append((torch.empty(sp["trials"], dtype=torch.int64, device="cuda"),
                     torch.empty(sp["trials"], dtype=torch.int64, device="cuda")))
        upd = n * sp["trials"] * sp["steps"]
        updates += upd
        if rb["path"] == psa.PSA_PATH_DENSE:
            dense_jobs += 1
            dense_valu += ops_per_update(0.0, False) * upd
            enc = jobs[-1].info()["dense_encoding"]   # 1 int8, 2 two-bit, 3 one-bit
            fp4 = enc in (2, 3)
            # matrix work in int8-peak equivalents: 1- and 2-bit couplings run
            # as fp4 x fp4 at twice the int8 rate
            mfma_ops += 2.0 * n * n * sp["trials"] * sp["steps"] * (0.5 if fp4 else 1.0)
            # algorithmic bytes per step: the encoded couplings once per
            # 64-trial tile, the spins (fp4 or int8) read and written once
            np_ = (n + 255) // 256 * 256 if fp4 else (n + 127) // 128 * 128
            tiles = (sp["trials"] + 63) // 64
            dense_bytes += (np_ * np_ * {1: 1.0, 2: 0.25, 3: 0.125}[enc] * tiles
                            + 2 * n * sp["trials"] * (0.5 if fp4 else 1.0)) * sp["steps"]
        else:
            valu_ops += ops_per_update(info["nnz"] / n * edge_ops(jobs[-1].info()), False) * upd
    S = max(sp["steps"] for sp in specs)

    def batched(ev=None):
        for j in jobs:
            j.reset()
        if ev is not None:
            ev[0].record(stream)
        psa.jobs_step_batch(ctx, jobs, S)
        if ev is not None:
            ev[1].record(stream)
        psa.jobs_energy_cut(ctx, jobs, [E for E, _ in outs], [C for _, C in outs])

    def sequential():
        for j, (E, C) in zip(alone, outs):
            j.reset()
            j.step(S)
            j.energy_cut(E, C)

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    ctx.timing()                     # clear
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        batched(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_timing(False)
    fam = ctx.timing()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    cuts_batched = [c.cpu().numpy().copy() for _, c in outs]
    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0
    same = all(np.array_equal(a, c.cpu().numpy()) for a, (_, c) in zip(cuts_batched, outs))
    value = updates * args.steps / wall
    # per-family device time per batch (each measured on its own stream)
    dense_ms = fam["dense_ms"] / args.steps
    batch_ms = fam["batch_ms"] / args.steps
    dense_frac = {
        "mfma": (mfma_ops / (dense_ms * 1e-3) / 1e12 / MFMA_I8_PEAK_TOPS) if dense_ms else 0.0,
        "alu": (dense_valu / (dense_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS) if dense_ms else 0.0,
        "hbm": (dense_bytes / (dense_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if dense_ms else 0.0,
    }
    if dense_ms >= batch_ms:
        bound = max(dense_frac, key=dense_frac.get)
        achieved = {"mfma": mfma_ops / (dense_ms * 1e-3) / 1e12,
                    "alu": dense_valu / (dense_ms * 1e-3) / 1e12,
                    "hbm": dense_bytes / (dense_ms * 1e-3) / 1e9}[bound]
        peak = {"mfma": MFMA_I8_PEAK_TOPS, "alu": VALU_PEAK_TOPS, "hbm": HBM_PEAK_GBS}[bound]
        roof = {"bound": bound, "kernel": "dense_step_kernel", "achieved": achieved,
                "peak": peak, "unit": "GB/s" if bound == "hbm" else "TOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel_ms": dense_ms / max(fam["dense_launches"] / args.steps, 1),
                "launches_per_batch": fam["dense_launches"] / args.steps,
                "dense_fracs": dense_frac}
    else:
        achieved = valu_ops / (batch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "anneal_batch_kernel", "achieved": achieved,
                "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": None, "kernel_ms": batch_ms, "dense_fracs": dense_frac}
    roof.update({"dense_ms_per_batch": dense_ms, "csr_batch_ms_per_batch": batch_ms,
                 "batch_span_ms": kernel_ms})
    line = {
        "metric": "p-bit updates/s (n x trials x steps / s), 1 GPU",
        "value": value,
        "unit": "p-bit updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 spins / int32 field / f32 pre-activation",
        "data": "synthetic",
        "config": {
            "workload": "c4", "graphs": len(specs), "trials": 64, "sweeps": S,
            "updates_per_batch": updates, "dense_path_jobs": dense_jobs,
            "tune_classes": psa.tune_cache_size(ctx), "tune_s": t_tune,
            "one_graph_at_a_time_updates_per_s": updates / wall_seq,
            "batched_over_one_at_a_time": wall_seq / (wall / args.steps),
            "identical_cuts": same,
        },
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        sample = []
        for sp in specs[:16]:
            n, u, v, w = inputs.make_graph(sp["graph"])
            sample.append((n, u, v, w, sp["seed"]))
        line["cpu_baseline"] = cpu_baseline_batch(sample, S, specs[0]["trials"])
    print(json.dumps(line), flush=True)


def bench_dense(args):
    """The dense step alone: 48 G(n, p) graphs, n ~ U{2000..4000}, p ~ U[0.04, 0.1],
    +1 weights (1-bit couplings; +-1 and 2-bit with --dense-weights pm1), 64 trials each, all on the matrix-core path,
    advanced together (one launch per step); 20 warm-up steps, then
    --steps x 30 steps timed with HIP events on the dense stream.  Reports
    the dense step's fractions of the matrix-core, vector and HBM peaks."""
    import torch
    from paper_2601_14476_amd import inputs, psa
    torch.cuda.set_device(0)
    rng = np.random.default_rng(7)
    specs = []
    for g in range(48):
        n = int(rng.integers(2000, 4000))
        p = float(rng.uniform(0.04, 0.1))
        specs.append(inputs.erdos_renyi(n, p, 500 + g, weights=args.dense_weights))
    ctx = psa.Context(0)
    ctx.set_dense_launch(DENSE_LAUNCH[args.dense_launch])
    graphs = [psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True) for n, u, v, w in specs]
    jobs = [psa.Job(ctx, g, 1000, 64, i, path=psa.PSA_PATH_DENSE) for i, g in enumerate(graphs)]
    psa.jobs_step_batch(ctx, jobs, 20)
    ctx.synchronize()
    steps = 30 * args.steps
    ctx.timing()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    psa.jobs_step_batch(ctx, jobs, steps)
    ctx.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_timing(False)
    tm = ctx.timing()
    per_us = tm["dense_ms"] / steps * 1e3
    n_arr = np.array([sp[0] for sp in specs], float)
    npad = np.ceil(n_arr / 256) * 256
    upd = float(n_arr.sum() * 64)
    # +1 weights (every coupling -1): 1-bit couplings, +-1: 2-bit; fp4 x fp4
    # products against the fp4 matrix peak; bytes: the couplings once per
    # 64 trials, fp4 spins read and written
    one_bit = args.dense_weights == "one"
    mfma = (2 * n_arr ** 2 * 64).sum() / (per_us * 1e-6) / 1e12
    hbm = (npad ** 2 / (8 if one_bit else 4) + n_arr * 64).sum() / (per_us * 1e-6) / 1e9
    valu = ops_per_update(0.0, False) * upd / (per_us * 1e-6) / 1e12
    fr = {"mfma": mfma / MFMA_F4_PEAK_TOPS, "alu": valu / VALU_PEAK_TOPS, "hbm": hbm / HBM_PEAK_GBS}
    bound = max(fr, key=fr.get)
    line = {
        "metric": "p-bit updates/s (n x trials x steps / s), 1 GPU",
        "value": upd * steps / wall, "unit": "p-bit updates/s", "n_gpus": 1,
        "steps": steps, "warmup": 20, "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4 couplings (%s encoded) x fp4 spins -> f32 field (exact integers)"
                 % ("1-bit" if one_bit else "2-bit"),
        "data": "synthetic",
        "config": {"workload": "c4-dense", "graphs": 48, "trials": 64, "n_range": [2000, 4000],
                   "p_range": [0.04, 0.1], "weights": "+1" if one_bit else "+-1"},
        "roofline": {"bound": bound, "kernel": "dense_step_kernel",
                     "achieved": {"mfma": mfma, "alu": valu, "hbm": hbm}[bound],
                     "peak": {"mfma": MFMA_F4_PEAK_TOPS, "alu": VALU_PEAK_TOPS, "hbm": HBM_PEAK_GBS}[bound],
                     "unit": "GB/s" if bound == "hbm" else "TOP/s", "frac": fr[bound],
                     "traffic": measured_traffic("c4-dense", "dense_step_kernel") if one_bit else None,
                     "kernel_us_per_step": per_us, "dense_fracs": fr},
    }
    print(json.dumps(line), flush=True)
    for j in jobs:
        j.close()
    for g in graphs:
        g.close()
    ctx.close()


def _serve_graph(spec):
    """Worker of the serving benchmark's graph producer: one job's edge list."""
    from paper_2601_14476_amd import inputs
    return inputs.make_graph(spec["graph"])


def bench_serve(args, pool):
    """Poisson arrivals at --rate jobs/s for --duration s; per job n in
    [800, 20000] (random sparse G(n, m), degree 4-50, +-1 weights, the job's
    own seeded graph), steps in [1000, 10000], trials in [32, 256], sigma in
    {0, 0.05, 0.1, 0.2}.  A process pool generates the jobs' edge lists in
    arrival order ahead of the arrivals (a client submits each at its
    arrival time; any lag behind the schedule is reported).  Reports
    completed jobs/s, p50/p99 latency (submit to result), served p-bit
    updates/s, and -- on a sample of the served jobs rerun one at a time on
    the same GPU, each tuned for running alone -- the one-at-a-time
    updates/s, with the cuts of every sampled trial compared (identical)."""
    import threading
    import torch
    from paper_2601_14476_amd import inputs, psa
    trace = inputs.serve_trace(rate=args.rate, duration=args.duration)
    # the producers' edge lists in arrival order, the first few seconds' worth
    # ready before the clock starts
    produced = pool.imap(_serve_graph, [sp for _, sp in trace], chunksize=1)
    ahead = []
    for _ in range(min(len(trace), int(4 * args.rate) + 8)):
        ahead.append(next(produced))
    torch.cuda.set_device(0)
    ctx = psa.Context(0)
    ctx.set_dense_launch(DENSE_LAUNCH[args.dense_launch])
    srv = psa.Server(ctx, max_resident=args.max_resident, quantum_steps=args.quantum)
    tickets = []
    updates = []
    lag = [0.0]
    t0 = time.perf_counter()

    def client():
        for idx, (at, spec) in enumerate(trace):
            if idx < len(ahead):
                n, u, v, w = ahead[idx]
            else:
                n, u, v, w = next(produced)
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            else:
                lag[0] = max(lag[0], -delay)
            tk = srv.submit(n, u, v, w, spec["steps"], spec["trials"], spec["seed"],
                            sigma_lambda=spec["sigma_lambda"], sigma_delta=spec["sigma_delta"],
                            sigma_nu=spec["sigma_nu"], p_mean=spec["p_mean"],
                            tune=not args.no_tune)
            tickets.append(tk)
            updates.append(n * spec["trials"] * spec["steps"])
            if idx < len(ahead):
                ahead[idx] = None

    th = threading.Thread(target=client)
    th.start()
    last = time.perf_counter()
    while th.is_alive():
        th.join(timeout=5.0)
        if time.perf_counter() - last > 20.0:
            st = srv.stats()
            print(f"[c5] {time.perf_counter() - t0:.0f}s submitted {len(tickets)}/{len(trace)} "
                  f"completed {st['completed']} resident {st['resident']} waiting {st['waiting']}",
                  file=sys.stderr, flush=True)
            last = time.perf_counter()
    pool.close()
    # progress while the queue drains (one line every ~20 s, whether or not
    # the job waited on has ended)
    for tk in tickets:
        while True:
            ended = True
            try:
                srv.wait(tk, timeout_s=5.0)
            except psa.PsaError as e:
                if e.status != psa.PSA_ETIMEDOUT:
                    raise
                ended = False
            if time.perf_counter() - last > 20.0:
                st = srv.stats()
                print(f"[c5] {time.perf_counter() - t0:.0f}s completed {st['completed']}/"
                      f"{len(tickets)} resident {st['resident']} waiting {st['waiting']}",
                      file=sys.stderr, flush=True)
                last = time.perf_counter()
            if ended:
                break
    print(f"[c5] drained at {time.perf_counter() - t0:.0f}s; one-at-a-time sample next",
          file=sys.stderr, flush=True)
    lat = []
    first_submit, last_end = None, 0
    done = 0
    cuts = {}
    for j, tk in enumerate(tickets):
        r, (_, _, C) = srv.result(tk)
        if r.status == psa.PSA_JOB_DONE:
            done += 1
            lat.append((r.end_us - r.submit_us) / 1e6)
            first_submit = r.submit_us if first_submit is None else min(first_submit, r.submit_us)
            last_end = max(last_end, r.end_us)
            cuts[j] = C
    stats = srv.stats()
    srv.close()
    makespan = (last_end - first_submit) / 1e6
    lat = np.array(lat)
    served = float(sum(updates) / makespan)
    # one at a time: a sample across the trace, each alone and tuned alone
    sample = sorted(cuts)[:: max(1, len(cuts) // max(1, args.alone_sample))][: args.alone_sample]
    alone_upd, alone_s, same = 0, 0.0, True
    for si, j in enumerate(sample):
        print(f"[c5] alone {si + 1}/{len(sample)}: job {j}", file=sys.stderr, flush=True)
        spec = trace[j][1]
        n, u, v, w = _serve_graph(spec)
        g = psa.Graph.from_edges(ctx, n, u, v, w, maxcut=True)
        kw = dict(sigma_lambda=spec["sigma_lambda"], sigma_delta=spec["sigma_delta"],
                  sigma_nu=spec["sigma_nu"], p_mean=spec["p_mean"])
        psa.tune_get(ctx, g, spec["steps"], spec["trials"], spec["seed"], **kw)
        ctx.synchronize()
        ta = time.perf_counter()
        _, _, C = psa.anneal(ctx, g, spec["steps"], spec["trials"], spec["seed"], spins=False,
                             tune=True, **kw)
        alone_s += time.perf_counter() - ta
        alone_upd += n * spec["trials"] * spec["steps"]
        same = same and bool(np.array_equal(C, cuts[j]))
        g.close()
    ctx.close()
    line = {
        "metric": "served jobs/s (p50/p99 latency), 1 GPU",
        "value": done / makespan,
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": len(tickets),
        "warmup": 0,
        "ms_per_step": makespan / max(done, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 spins / int32 field / f32 pre-activation",
        "data": "synthetic",
        "config": {
            "workload": "c5", "arrival_rate": args.rate, "duration_s": args.duration,
            "jobs": len(tickets), "completed": done, "failed": stats["failed"],
            "quantum_steps": args.quantum, "max_resident": args.max_resident,
            "graphs": "each job's own seeded G(n, m)",
            "submit_lag_max_s": lag[0],
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()),
            "served_updates_per_s": served,
            "offered_updates_per_s": float(sum(updates) / args.duration),
            "makespan_s": makespan, "quanta": stats["quanta"],
            "peak_resident": stats["peak_resident"],
            "autotuned": not args.no_tune,
            "alone_sample_jobs": len(sample),
            "alone_updates_per_s": alone_upd / alone_s if alone_s > 0 else None,
            "served_vs_alone": served / (alone_upd / alone_s) if alone_s > 0 else None,
            "alone_cuts_identical": same,
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
