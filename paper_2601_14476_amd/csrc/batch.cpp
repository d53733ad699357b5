// batch.cpp -- many runs of uneven size in one launch.
//
// psa_jobs_step_batch advances a set of existing jobs by up to k steps each
// with one launch of the batch kernel: a work list holds one item per
// (job, trial); each workgroup reads its job's arguments from a device table
// and runs the kernel variant that job needs.  Work items are placed so that
// a job's workgroups land on one XCD (workgroups are dispatched to the eight
// XCDs round-robin by index), heaviest jobs first.  psa_anneal_batch wraps it:
// create the jobs, run them to the end, write energies, cuts and spins.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "engine.hpp"
#include "psa.h"

using psa::set_error;

namespace {

constexpr int kXcds = 8;
constexpr int kChunk = 16;  // work items placed on one XCD together


// Grow-only device buffer kept by the context between batched launches.
psa_status ensure(void **buf, size_t *cap, size_t bytes) {
    if (*cap >= bytes) return PSA_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc(buf, bytes) != hipSuccess) {
        *buf = nullptr;
        set_error("batch: device allocation failed");
        return PSA_ENOMEM;
    }
    *cap = bytes;
    return PSA_OK;
}

}  // namespace

namespace psa {

// Build the XCD-aware work list for `jobs` (cost = trials * n4 * steps).
void build_work_list(const std::vector<int32_t> &trials, const std::vector<double> &cost,
                     std::vector<int2> *work) {
    struct Chunk {
        int32_t job, q0, q1;
        double cost;
    };
    std::vector<Chunk> chunks;
    for (size_t j = 0; j < trials.size(); ++j) {
        const double per = trials[j] > 0 ? cost[j] / trials[j] : 0.0;
        for (int32_t q = 0; q < trials[j]; q += kChunk) {
            const int32_t q1 = std::min(trials[j], q + kChunk);
            chunks.push_back(Chunk{static_cast<int32_t>(j), q, q1, per * (q1 - q)});
        }
    }
    std::stable_sort(chunks.begin(), chunks.end(),
                     [](const Chunk &a, const Chunk &b) { return a.cost > b.cost; });
    std::vector<std::vector<int2>> queue(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (const Chunk &c : chunks) {
        const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        for (int32_t q = c.q0; q < c.q1; ++q) queue[x].push_back(make_int2(c.job, q));
        load[x] += c.cost;
    }
    size_t len = 0;
    for (const auto &qu : queue) len = std::max(len, qu.size());
    work->assign(len * kXcds, make_int2(-1, 0));
    for (int x = 0; x < kXcds; ++x)
        for (size_t s = 0; s < queue[x].size(); ++s) (*work)[s * kXcds + x] = queue[x][s];
}

// Automatic path choice.  Whole-device estimates per step (above the floors
// below): the CSR walk issues ~60 + 3 d lane-operations per update (d = mean
// degree) at 39.3 T lane-ops/s; the dense product costs 2 np^2 tp operations
// at half the int8 (or, 1- and 2-bit couplings, fp4) matrix peak, or the
// bytes of J once per trial tile at the HBM peak, whichever is larger, plus
// ~60 lane-operations of epilogue per update.
// Latency floors of a step: the CSR sweep's step is a barrier and a chain of
// LDS reads inside one persistent launch; the dense step is a launch of its
// own.  They decide for small runs, whose throughput terms are tiny (a G1-
// sized run of 10 trials: 2 us per CSR step measured, several times that per
// dense step).
constexpr double kCsrStepFloorSeconds = 1.5e-6;
constexpr double kDenseStepFloorSeconds = 6.0e-6;

double csr_step_seconds(const DevGraph &g, const DevRun &run, const AnnealPlan &plan) {
    // lane-ops per update: RNG, activation and decision (about 60), plus a
    // gather per edge: a few ops from LDS, tens when the rows stream from
    // memory (latency-bound gathers of one trial per workgroup)
    const double d = g.nnz / static_cast<double>(std::max(g.n, 1));
    const double per_edge = plan.csr_lds ? 3.0 : 40.0;
    return std::max(kCsrStepFloorSeconds,
                    static_cast<double>(g.n) * run.t4 * (60.0 + per_edge * d) / kValuOpsPerSecond);
}

double dense_step_seconds(int32_t n, int32_t t4, bool two_bit, bool one_bit) {
    two_bit = two_bit || one_bit;
    const double np = two_bit ? (n + 255) / 256 * 256 : (n + 127) / 128 * 128;
    const int32_t nb = t4 >= 64 ? 4 : (t4 >= 32 ? 2 : 1);
    const double tp = std::ceil(t4 / (16.0 * nb)) * 16.0 * nb;
    const double mfma = 2.0 * np * np * tp / (0.5 * (two_bit ? kMfmaF4OpsPerSecond : kMfmaI8OpsPerSecond));
    const double bytes = np * np * (one_bit ? 0.125 : (two_bit ? 0.25 : 1.0)) * (tp / (16.0 * nb)) / kHbmBytesPerSecond;
    return kDenseStepFloorSeconds + std::max(mfma, bytes) + static_cast<double>(n) * t4 * 60.0 / kValuOpsPerSecond;
}

bool dense_two_bit(const psa_graph *g) {
    int32_t mag = 0;
    for (int32_t v : g->val_host) {
        const int32_t a = v < 0 ? -v : v;
        if (a == 0) return false;
        if (mag == 0) mag = a;
        if (a != mag) return false;
    }
    return true;
}

bool dense_one_bit(const psa_graph *g) {
    if (g->val_host.empty() || g->val_host[0] == 0) return false;
    return std::all_of(g->val_host.begin(), g->val_host.end(), [&](int32_t v) { return v == g->val_host[0]; });
}

bool prefer_dense(const psa_graph *g, const DevRun &run, const AnnealPlan &plan) {
    if (g->info.n < 256) return false;
    const bool two_bit = dense_two_bit(g);
    if (!two_bit && std::any_of(g->val_host.begin(), g->val_host.end(),
                                [](int32_t v) { return v < -127 || v > 127; }))
        return false;
    return dense_step_seconds(g->info.n, run.t4, two_bit, dense_one_bit(g)) < 0.7 * csr_step_seconds(g->dev, run, plan);
}

// Work list of the dense runs `idx` of `table` (one encoding): items (job,
// 256-row group, trial tile) in chunks of up to 16 items -- consecutive row
// groups, each with its trial tiles next to each other -- each chunk given
// whole to the least loaded of the 8 XCDs, heaviest runs first.  Workgroup b
// of a launch runs on XCD b % 8, so slot b takes item b / 8 of that XCD's
// queue (or an empty slot): a chunk's items share their spin tiles in one L2,
// and the trial tiles of a row group read its couplings at about the same
// time there.
static void dense_work_list(const std::vector<DenseJob> &table, const std::vector<int32_t> &idx,
                            int32_t nb, std::vector<int4> *out) {
    constexpr int32_t kXcd = 8, kChunk = 16;
    std::vector<int32_t> order(idx);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const DenseJob &x = table[a], &y = table[b];
        return static_cast<double>(x.np) * x.np * x.tp > static_cast<double>(y.np) * y.np * y.tp;
    });
    std::vector<std::vector<int4>> bins(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int32_t j : order) {
        const DenseJob &d = table[j];
        const int32_t groups = (d.np + 255) / 256, tiles = d.tp / (16 * nb);
        const int32_t span = std::max(1, kChunk / tiles);  // row groups per chunk
        for (int32_t g0 = 0; g0 < groups; g0 += span) {
            const int32_t g1 = std::min(groups, g0 + span);
            const int32_t x = static_cast<int32_t>(std::min_element(load.begin(), load.end()) - load.begin());
            for (int32_t g = g0; g < g1; ++g)
                for (int32_t tt = 0; tt < tiles; ++tt) bins[x].push_back(make_int4(j, g, tt, 0));
            load[x] += static_cast<double>(g1 - g0) * tiles * d.np;
        }
    }
    size_t len = 0;
    for (const auto &b : bins) len = std::max(len, b.size());
    out->assign(len * kXcd, make_int4(-1, 0, 0, 0));
    for (int32_t x = 0; x < kXcd; ++x)
        for (size_t q = 0; q < bins[x].size(); ++q) (*out)[q * kXcd + x] = bins[x][q];
}

// One dense step sequence on stream s, launched step by step: replayed from a
// captured graph of the same shape, captured now (evicting the least recently
// used graph past kDenseGraphCache, after the stream has drained), or --
// use_graph false, or a single step -- launched one by one.  *graph: it ran
// as a graph.
static psa_status dense_sequence(psa_ctx *ctx, hipStream_t s, const DenseJob *table, const int4 *work,
                                 int32_t nwork, int32_t nb, int32_t enc, int32_t mode, int32_t steps,
                                 bool use_graph, bool *graph) {
    *graph = false;
    if (!use_graph || steps < kDenseGraphMinSteps) {
        PSA_HIP(launch_dense_steps(s, table, work, nwork, nb, enc, mode, steps), "dense step launch");
        return PSA_OK;
    }
    auto &cache = ctx->dense_graph_cache;
    auto it = std::find_if(cache.begin(), cache.end(), [&](const DenseGraph &d) {
        return d.table == table && d.work == work && d.nwork == nwork && d.nb == nb && d.enc == enc &&
               d.mode == mode && d.steps == steps;
    });
    if (it == cache.end()) {
        PSA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        const hipError_t le = launch_dense_steps(s, table, work, nwork, nb, enc, mode, steps);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(s, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            PSA_HIP(le != hipSuccess ? le : ce, "dense step capture");
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        PSA_HIP(ie, "hipGraphInstantiate");
        if (cache.size() >= kDenseGraphCache) {
            PSA_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
            (void)hipGraphExecDestroy(cache.front().exec);
            cache.erase(cache.begin());
        }
        cache.push_back(DenseGraph{table, work, nwork, nb, enc, mode, steps, exec});
        it = cache.end() - 1;
    } else {
        std::rotate(it, it + 1, cache.end());  // most recently used last
        it = cache.end() - 1;
    }
    PSA_HIP(hipGraphLaunch(it->exec, s), "hipGraphLaunch");
    *graph = true;
    return PSA_OK;
}

// Task list of the persistent launch: whole runs dealt to kDenseQueues queues
// (heaviest first, each to the least loaded queue), each queue's items run by
// run (256-row group, then trial tile), no empty slots; q->off the queues'
// bounds in the list.
static void dense_task_list(const std::vector<DenseJob> &table, const std::vector<int32_t> &idx, int32_t nb,
                            std::vector<int4> *out, DenseQueues *q) {
    std::vector<int32_t> order(idx);
    auto cost = [&](int32_t j) { return static_cast<double>(table[j].np) * table[j].np * table[j].tp; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    std::vector<std::vector<int32_t>> queue(kDenseQueues);
    std::vector<double> load(kDenseQueues, 0.0);
    for (int32_t j : order) {
        const int32_t x = static_cast<int32_t>(std::min_element(load.begin(), load.end()) - load.begin());
        queue[x].push_back(j);
        load[x] += cost(j);
    }
    out->clear();
    for (int32_t x = 0; x < kDenseQueues; ++x) {
        q->off[x] = static_cast<int32_t>(out->size());
        for (int32_t j : queue[x]) {
            const DenseJob &d = table[j];
            const int32_t groups = (d.np + 255) / 256, tiles = d.tp / (16 * nb);
            for (int32_t g = 0; g < groups; ++g)
                for (int32_t tt = 0; tt < tiles; ++tt) out->push_back(make_int4(j, g, tt, 0));
        }
    }
    q->off[kDenseQueues] = static_cast<int32_t>(out->size());
}

psa_status dense_step_jobs(psa_ctx *ctx, psa_job *const *jobs, int32_t count, int32_t k, double share) {
    std::vector<psa::DenseJob> table;
    std::vector<psa_job *> live;
    constexpr int kE = kDenseEncodings;
    std::vector<int32_t> by_enc[kE];
    int32_t max_steps = 0, nb[kE] = {4, 4, 4};
    bool plain[kE] = {true, true, true};     // every run of the encoding is plain pSA
    bool identity[kE] = {true, true, true};  // ... with identity factors and no gate
    for (int32_t j = 0; j < count; ++j) {
        psa_job *job = jobs[j];
        const psa_graph *g = job->g;
        const int32_t te = static_cast<int32_t>(std::min<int64_t>(int64_t{job->t} + k, job->run.steps));
        if (te <= job->t) continue;
        psa::DenseJob d;
        d.n = g->info.n;
        d.n4 = g->dev.n4;
        d.np = g->np;
        d.t4 = job->run.t4;
        d.tp = job->tp;
        d.t = job->t;
        d.t_end = te;
        d.scale = g->dense_scale;
        d.items = 0;
        d.J = g->d_dense;
        d.m0 = job->d_m;
        d.m1 = job->d_m + static_cast<size_t>(job->tp) * g->np;
        d.h = g->dev.h;
        d.i0 = job->run.i0;
        d.lam = job->run.lambda;
        d.dlt = job->run.delta;
        d.thr = job->run.thr24;
        d.k0 = job->run.key0;
        d.k1 = job->run.key1;
        d.xs = job->run.xs;
        d.stall24 = job->run.stall24;
        d.ring = job->run.ring;
        d.alpha = job->run.alpha;
        d.t_res = job->run.t_res;
        const int32_t e = g->dense_enc;
        plain[e] = plain[e] && d.xs == nullptr && d.ring == nullptr && d.t_res == 0;
        identity[e] = identity[e] && job->identity_factors;
        by_enc[e].push_back(static_cast<int32_t>(table.size()));
        nb[e] = std::min(nb[e], job->plan.nb);
        table.push_back(d);
        live.push_back(job);
        max_steps = std::max(max_steps, (te - job->t) * std::max(job->run.t_res, 1));
    }
    if (live.empty()) return PSA_OK;
    // fp4 couplings: trial tiles of at most 32 trials.  The two tiles of a
    // 64-trial row group read the same couplings (the second mostly from L2,
    // the work list keeping them together), and twice the items per launch
    // both outnumber the resident workgroup slots, so that items start in
    // waves and their coupling and epilogue phases overlap, and even out the
    // items per compute unit in the vector-bound epilogue (48 runs of n
    // 2,000-4,000 at 64 trials, 1-bit couplings: 25.1-25.5 against 26.8-26.9
    // us per step, the second tile's coupling reads adding 4.5 MB of HBM
    // traffic to 70 MB; 16-trial tiles 30.7 us; 2-bit couplings 32.5 us
    // either way).
    for (int e = 0; e < kE; ++e)
        if (dense_fp4(e)) nb[e] = std::min(nb[e], 2);
    const int32_t how = max_steps >= kDenseGraphMinSteps ? ctx->dense_launch : kDenseLaunchSteps;
    std::vector<int4> work, part;
    size_t off[kE] = {0, 0, 0}, len[kE] = {0, 0, 0};
    DenseQueues queues[kE] = {};
    for (int e = 0; e < kE; ++e) {
        if (by_enc[e].empty()) continue;
        if (how == kDenseLaunchPersistent && plain[e])
            dense_task_list(table, by_enc[e], nb[e], &part, &queues[e]);
        else
            dense_work_list(table, by_enc[e], nb[e], &part);
        off[e] = work.size();
        len[e] = part.size();
        work.insert(work.end(), part.begin(), part.end());
    }
    for (const int4 &w : work)
        if (w.x >= 0) ++table[static_cast<size_t>(w.x)].items;
    PSA_HIP(hipStreamSynchronize(ctx->stream2), "hipStreamSynchronize");
    if (ctx->h_dense_err && (ctx->h_dense_err[0] | ctx->h_dense_err[1] | ctx->h_dense_err[2])) {
        ctx->h_dense_err[0] = ctx->h_dense_err[1] = ctx->h_dense_err[2] = 0u;
        set_error("dense step sequence: a workgroup waited past its limit for another work item of its run; "
                  "the spins of that quantum are not valid");
        return PSA_EHIP;
    }
    psa_status st;
    if ((st = ensure(&ctx->d_dense_table, &ctx->dense_table_cap, table.size() * sizeof(psa::DenseJob))) != PSA_OK)
        return st;
    if ((st = ensure(&ctx->d_dense_work, &ctx->dense_work_cap, work.size() * sizeof(int4))) != PSA_OK)
        return st;
    const int32_t sync_words = dense_sync_words(static_cast<int32_t>(table.size()));
    if (how == kDenseLaunchPersistent) {
        void *p = ctx->d_dense_sync;
        if ((st = ensure(&p, &ctx->dense_sync_cap, kE * static_cast<size_t>(sync_words) * sizeof(uint32_t))) !=
            PSA_OK)
            return st;
        ctx->d_dense_sync = static_cast<uint32_t *>(p);
        if (!ctx->h_dense_err) {
            void *h = nullptr;
            PSA_HIP(hipHostMalloc(&h, kE * sizeof(uint32_t), hipHostMallocDefault), "hipHostMalloc");
            ctx->h_dense_err = static_cast<uint32_t *>(h);
            ctx->h_dense_err[0] = ctx->h_dense_err[1] = ctx->h_dense_err[2] = 0u;
        }
    }
    ctx->h_dense_table = table;
    ctx->h_dense_work = work;
    for (psa_job *job : live)
        for (int half = 0; half < 2; ++half)  // both buffers: a fully defined state
            PSA_HIP(psa::launch_to_dense(ctx->stream2, job->g->dense_enc, job->g->info.n, job->run.t4, job->g->np,
                                         job->tp, job->d_spins,
                                         job->d_m + static_cast<size_t>(half) * job->tp * job->g->np),
                    "dense layout");
    PSA_HIP(hipMemcpyAsync(ctx->d_dense_table, ctx->h_dense_table.data(),
                           table.size() * sizeof(psa::DenseJob), hipMemcpyHostToDevice, ctx->stream2),
            "dense table upload");
    PSA_HIP(hipMemcpyAsync(ctx->d_dense_work, ctx->h_dense_work.data(), work.size() * sizeof(int4),
                           hipMemcpyHostToDevice, ctx->stream2),
            "dense work upload");
    const int4 *dwork = static_cast<const int4 *>(ctx->d_dense_work);
    const psa::DenseJob *dtable = static_cast<const psa::DenseJob *>(ctx->d_dense_table);
    hipEvent_t ev = nullptr;
    if ((st = time_begin(ctx, ctx->stream2, &ev)) != PSA_OK) return st;
    int64_t launches = 0, replayed = 0;
    // launched step by step, the sequences of a second (and third) encoding
    // run on the third stream beside the first encoding's: a few runs of one
    // encoding take latency-bound steps that would otherwise follow the
    // other encoding's whole sequence (in a mix of 256 graphs, 24 runs of
    // 2-bit couplings took 15 ms per 1,000 steps alone, 127 runs of 1-bit
    // ones 62-64 ms, and the two 72.7 ms side by side)
    int32_t present = 0;
    for (int e = 0; e < kE; ++e) present += len[e] > 0 ? 1 : 0;
    const bool side = how == kDenseLaunchSteps && present > 1;
    if (side) {
        PSA_HIP(hipEventRecord(ctx->ev_fork3, ctx->stream2), "hipEventRecord");
        PSA_HIP(hipStreamWaitEvent(ctx->stream3, ctx->ev_fork3, 0), "hipStreamWaitEvent");
    }
    bool first = true;
    for (int e = 0; e < kE; ++e) {
        if (len[e] == 0) continue;
        const int32_t enc = e;
        const int32_t mode = plain[e] ? (identity[e] ? 2 : 1) : 0;
        if (how == kDenseLaunchPersistent && mode != 0) {
            uint32_t *sync = ctx->d_dense_sync + static_cast<size_t>(e) * sync_words;
            const int32_t cus = std::clamp(static_cast<int32_t>(std::lround(share * ctx->num_cu)), kDenseQueues,
                                           ctx->num_cu);
            PSA_HIP(psa::launch_dense_persistent(ctx->stream2, dtable, dwork + off[e], queues[e], nb[e], enc, mode,
                                                 max_steps, sync, sync_words, ctx->dense_max_polls, cus),
                    "dense step sequence launch");
            PSA_HIP(hipMemcpyAsync(ctx->h_dense_err + e, sync + 32 * kDenseQueues, sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, ctx->stream2),
                    "dense step error flag");
            launches += 1;
            continue;
        }
        bool graph = false;
        hipStream_t s = side && !first ? ctx->stream3 : ctx->stream2;
        first = false;
        if ((st = dense_sequence(ctx, s, dtable, dwork + off[e], static_cast<int32_t>(len[e]), nb[e], enc, mode,
                                 max_steps, how == kDenseLaunchGraph, &graph)) != PSA_OK)
            return st;
        launches += max_steps;
        replayed += graph ? max_steps : 0;
    }
    if (side) {
        PSA_HIP(hipEventRecord(ctx->ev_join3, ctx->stream3), "hipEventRecord");
        PSA_HIP(hipStreamWaitEvent(ctx->stream2, ctx->ev_join3, 0), "hipStreamWaitEvent");
    }
    if (ev) ctx->timed_graph_launches += replayed;
    if ((st = time_end(ctx, ctx->stream2, kTimeDense, ev, launches)) != PSA_OK) return st;
    for (size_t j = 0; j < live.size(); ++j) {
        psa_job *job = live[j];
        const psa::DenseJob &d = table[j];
        const int8_t *fin = (((d.t_end - d.t) * std::max(d.t_res, 1)) & 1) ? d.m1 : d.m0;
        PSA_HIP(psa::launch_from_dense(ctx->stream2, job->g->dense_enc, job->g->info.n, job->run.t4, job->g->np, fin,
                                       job->d_spins),
                "dense layout");
        job->t = d.t_end;
    }
    return PSA_OK;
}

}  // namespace psa

extern "C" {

psa_status psa_jobs_step_batch(psa_ctx *ctx, int32_t count, psa_job *const *jobs, int32_t k) {
    return psa::guarded("psa_jobs_step_batch", [&]() -> psa_status {
        if (!ctx || count < 0 || (count > 0 && !jobs) || k < 0) {
            set_error("psa_jobs_step_batch: invalid arguments");
            return PSA_EINVAL;
        }
        std::vector<psa::BatchJob> table;
        std::vector<int32_t> trials;
        std::vector<double> cost;
        std::vector<int32_t> t_end;
        std::vector<psa_job *> dense_jobs;
        size_t lds = 0;
        int32_t max_lanes = 0;
        double dense_s = 0.0, csr_s = 0.0;  // model estimates of the two families' device time
        for (int32_t j = 0; j < count; ++j) {
            psa_job *job = jobs[j];
            if (!job || job->ctx != ctx) {
                set_error("psa_jobs_step_batch: job " + std::to_string(j) + " is NULL or belongs to "
                          "another context");
                return PSA_EINVAL;
            }
            for (int32_t i = 0; i < j; ++i)
                if (jobs[i] == job) {
                    set_error("psa_jobs_step_batch: job listed twice");
                    return PSA_EINVAL;
                }
            const int32_t te = static_cast<int32_t>(
                std::min<int64_t>(int64_t{job->t} + k, job->run.steps));
            t_end.push_back(te);
            if (te <= job->t) continue;
            if (job->plan.dense) {
                dense_jobs.push_back(job);
                dense_s += psa::dense_step_seconds(job->g->info.n, job->run.t4, job->g->dense_enc == psa::kDenseT2,
                                                   job->g->dense_enc == psa::kDenseB1) *
                           (te - job->t);
                continue;
            }
            psa::AnnealPlan plan;
            int32_t variant = 0;
            std::string why;
            if (!psa::plan_batch_item(job->g->dev, job->run, job->plan.tpw,
                                      job->plan.tpw == 1 ? job->plan.lpt : 0, ctx->max_lds, &plan,
                                      &variant, &why)) {
                set_error("psa_jobs_step_batch: " + why);
                return PSA_EUNSUPPORTED;
            }
            csr_s += psa::csr_step_seconds(job->g->dev, job->run, plan) * (te - job->t);
            psa::BatchJob bj;
            psa::fill_anneal_args(&bj.a, job->g->dev, job->run, job->d_order, job->t, te);
            bj.variant = variant;
            table.push_back(bj);
            trials.push_back(plan.tpw == 4 ? job->run.t4 / 4 : job->run.trials);  // work items
            cost.push_back(static_cast<double>(job->run.trials) * job->g->dev.n4 * (te - job->t));
            lds = std::max(lds, plan.lds_bytes);
            max_lanes = std::max(max_lanes, job->g->dev.n4 / 4 * plan.lpt);
        }
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        if (!dense_jobs.empty()) {
            // dense runs on the second stream, concurrently with the CSR launch
            PSA_HIP(hipEventRecord(ctx->ev_fork, ctx->stream), "hipEventRecord");
            PSA_HIP(hipStreamWaitEvent(ctx->stream2, ctx->ev_fork, 0), "hipStreamWaitEvent");
            // a persistent dense launch keeps its workgroups resident: it gets
            // the dense family's modelled share of the device
            const double share = csr_s > 0.0 ? dense_s / (dense_s + csr_s) : 1.0;
            psa_status st = psa::dense_step_jobs(ctx, dense_jobs.data(),
                                                 static_cast<int32_t>(dense_jobs.size()), k, share);
            if (st != PSA_OK) return st;
            PSA_HIP(hipEventRecord(ctx->ev_join, ctx->stream2), "hipEventRecord");
        }
        if (table.empty()) {
            if (!dense_jobs.empty())
                PSA_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0), "hipStreamWaitEvent");
            return PSA_OK;
        }
        std::vector<int2> work;
        psa::build_work_list(trials, cost, &work);
        // the staging buffers are reused: the previous batched launch must be done
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        psa_status st;
        if ((st = ensure(&ctx->d_batch_table, &ctx->batch_table_cap,
                         table.size() * sizeof(psa::BatchJob))) != PSA_OK)
            return st;
        if ((st = ensure(&ctx->d_batch_work, &ctx->batch_work_cap, work.size() * sizeof(int2))) != PSA_OK)
            return st;
        ctx->h_batch_table = table;
        ctx->h_batch_work = work;
        PSA_HIP(hipMemcpyAsync(ctx->d_batch_table, ctx->h_batch_table.data(),
                               table.size() * sizeof(psa::BatchJob), hipMemcpyHostToDevice, ctx->stream),
                "batch table upload");
        PSA_HIP(hipMemcpyAsync(ctx->d_batch_work, ctx->h_batch_work.data(), work.size() * sizeof(int2),
                               hipMemcpyHostToDevice, ctx->stream),
                "batch work upload");
        const int32_t block = max_lanes > 1024 ? 1024 : (max_lanes > 256 ? 512 : 256);
        hipEvent_t ev = nullptr;
        if ((st = psa::time_begin(ctx, ctx->stream, &ev)) != PSA_OK) return st;
        PSA_HIP(psa::launch_anneal_batch(ctx->stream, static_cast<const psa::BatchJob *>(ctx->d_batch_table),
                                         static_cast<const int2 *>(ctx->d_batch_work),
                                         static_cast<int32_t>(work.size()), block, lds),
                "batch anneal launch");
        if ((st = psa::time_end(ctx, ctx->stream, psa::kTimeBatch, ev, 1)) != PSA_OK) return st;
        for (int32_t j = 0; j < count; ++j) jobs[j]->t = std::max(jobs[j]->t, t_end[j]);
        if (!dense_jobs.empty())
            PSA_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0), "hipStreamWaitEvent");
        return PSA_OK;
    });
}

psa_status psa_anneal_batch(psa_ctx *ctx, int32_t count, const psa_batch_item *items,
                            uint32_t flags) {
    return psa::guarded("psa_anneal_batch", [&]() -> psa_status {
        if (!ctx || count < 0 || (count > 0 && !items) ||
            (flags & ~(PSA_OUT_DEVICE | PSA_BATCH_SEQUENTIAL)) != 0) {
            set_error("psa_anneal_batch: invalid arguments");
            return PSA_EINVAL;
        }
        for (int32_t j = 0; j < count; ++j)
            if (!items[j].graph || !items[j].energy_out || !items[j].cut_out) {
                set_error("psa_anneal_batch: item " + std::to_string(j) +
                          " needs a graph, energy_out and cut_out");
                return PSA_EINVAL;
            }
        std::vector<std::unique_ptr<psa_job, void (*)(psa_job *)>> owned;
        std::vector<psa_job *> jobs;
        int32_t max_steps = 0;
        for (int32_t j = 0; j < count; ++j) {
            psa_run_desc d = items[j].desc;
            if (!(flags & PSA_BATCH_SEQUENTIAL)) {
                if (d.flags & PSA_TUNE) {
                    psa_status st = psa::tuned_desc(ctx, items[j].graph, &d, PSA_TUNE_BATCH);
                    if (st != PSA_OK) {
                        set_error("psa_anneal_batch: item " + std::to_string(j) + ": " + psa_last_error());
                        return st;
                    }
                }
                if (d.trials_per_group == 0) d.trials_per_group = 1;
            }
            psa_job *job = nullptr;
            psa_status st = psa_job_create(ctx, items[j].graph, &d, &job);
            if (st != PSA_OK) {
                set_error("psa_anneal_batch: item " + std::to_string(j) + ": " + psa_last_error());
                return st;
            }
            owned.emplace_back(job, psa_job_destroy);
            jobs.push_back(job);
            max_steps = std::max(max_steps, d.steps);
        }
        psa_status st;
        if (flags & PSA_BATCH_SEQUENTIAL) {
            for (psa_job *job : jobs)
                if ((st = psa_job_step(job, job->run.steps)) != PSA_OK) return st;
        } else {
            if ((st = psa_jobs_step_batch(ctx, count, jobs.data(), max_steps)) != PSA_OK) return st;
        }
        const uint32_t out = flags & PSA_OUT_DEVICE;
        if (!(flags & PSA_BATCH_SEQUENTIAL)) {
            // the batch's read-outs in two launches
            std::vector<int64_t *> energy(static_cast<size_t>(count)), cut(static_cast<size_t>(count));
            for (int32_t j = 0; j < count; ++j) {
                energy[static_cast<size_t>(j)] = items[j].energy_out;
                cut[static_cast<size_t>(j)] = items[j].cut_out;
            }
            if ((st = psa_jobs_energy_cut(ctx, count, jobs.data(), energy.data(), cut.data(), out)) != PSA_OK)
                return st;
        }
        for (int32_t j = 0; j < count; ++j) {
            if ((flags & PSA_BATCH_SEQUENTIAL) &&
                (st = psa_job_energy_cut(jobs[j], items[j].energy_out, items[j].cut_out, out)) != PSA_OK)
                return st;
            if (items[j].spins_out &&
                (st = psa_job_read_spins(jobs[j], items[j].spins_out, out)) != PSA_OK)
                return st;
        }
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

}  // extern "C"
