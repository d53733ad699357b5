// tune.cpp -- measured choice of field path and launch shape.
//
// The cost model of the automatic path choice is a rough guide: the CSR
// sweep's speed depends on whether the edges fit in LDS, on row-length
// spread and on how many workgroups a run exposes, the dense path's on
// whether its coupling bytes stay in cache.  The autotuner settles the
// choice by timing scratch copies of the run on the device, per shape class
// of graph, and keeps the answer in the context.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"
#include "psa.h"

namespace psa {
namespace {

struct Candidate {
    uint32_t path;
    int32_t tpw, lpt;
};

using JobPtr = std::unique_ptr<psa_job, void (*)(psa_job *)>;

bool dense_encodable(const psa_graph *g) {
    if (dense_two_bit(g)) return true;
    return std::none_of(g->val_host.begin(), g->val_host.end(),
                        [](int32_t v) { return v < -127 || v > 127; });
}

// Shape class of a tuning problem: mode, trials, n within 1/8 octave, mean
// degree within 1/4 octave, dense encoding, rows short enough for 16-bit
// packing, update rule.
TuneKey tune_key(const psa_graph *g, int32_t trials, uint32_t mode, uint32_t algorithm) {
    const double n = std::max(g->info.n, 1);
    const double d = static_cast<double>(g->info.nnz) / n;
    const int64_t enc = dense_one_bit(g) ? 3 : (dense_two_bit(g) ? 2 : (dense_encodable(g) ? 1 : 0));
    // batched mode times copies of the run that fill the chip, so the trial
    // count matters by its magnitude: half-octave classes; alone, exactly
    const int64_t tkey = mode == PSA_TUNE_BATCH
                             ? static_cast<int64_t>(std::ceil(std::log2(std::max(trials, 1)) * 2.0))
                             : trials;
    return TuneKey{static_cast<int64_t>(mode), tkey, static_cast<int64_t>(std::ceil(std::log2(n) * 8.0)),
                   static_cast<int64_t>(std::floor(std::log2(1.0 + d) * 4.0)), enc,
                   g->dev.max_degree <= 255 ? 1 : 0, static_cast<int64_t>(algorithm)};
}

// Time one candidate: `copies` scratch runs of desc with the candidate's
// shape, stepped alone (one run) or batched.  *us = device microseconds per
// run and step; EUNSUPPORTED when the candidate does not apply.  A call that
// advances runs by k steps costs a + b k: a covers what every call does once
// (the dense path's layout conversions of every run, table uploads), b the
// steps.  Runs advance by a whole quantum or anneal per call, so the step
// cost b decides: it is taken from calls of `probe` and 2 `probe` steps, b =
// (T2 - T1) / probe, when the run has the steps for both (else T1 / probe).
// Timing short calls alone put the dense path's per-run conversions into
// every step (about 5x its per-step cost in a batch of 1,000 steps).
psa_status time_candidate(psa_ctx *ctx, const psa_graph *g, const psa_run_desc &base,
                          const Candidate &c, int32_t probe, uint32_t mode, double *us) {
    psa_run_desc d = base;
    d.flags = c.path;
    d.trials_per_group = c.tpw;
    d.lanes_per_task = c.lpt;
    d.block = 0;
    int32_t copies = 1;
    if (mode == PSA_TUNE_BATCH) {
        // enough copies that the batched launch fills the chip
        int64_t groups;
        if (c.path == PSA_PATH_DENSE) {
            // 256-row groups x trial tiles (32 trials with fp4 couplings)
            const int64_t tile = dense_two_bit(g) ? 32 : 64;
            groups = (g->info.n + 255) / 256 * ((d.trials + tile - 1) / tile);
        } else {
            groups = c.tpw == 4 ? (d.trials + 3) / 4 : d.trials;
        }
        copies = static_cast<int32_t>(std::clamp<int64_t>((2 * ctx->num_cu + groups - 1) / groups, 1, 16));
    }
    std::vector<JobPtr> owned;
    std::vector<psa_job *> jobs;
    // one run, then clones sharing its read-only arrays (every job waits for
    // the stream before it is freed, and none is launched after that)
    for (int32_t i = 0; i < copies; ++i) {
        psa_job *job = nullptr;
        const psa_status st = i == 0 ? psa_job_create(ctx, g, &d, &job)
                                     : clone_job_for_timing(jobs[0], &job);
        if (st != PSA_OK) return st;
        owned.emplace_back(job, psa_job_destroy);
        jobs.push_back(job);
    }
    const int32_t warm = base.steps > probe ? 1 : 0;
    auto advance = [&](int32_t k) -> psa_status {
        if (mode == PSA_TUNE_BATCH) return psa_jobs_step_batch(ctx, copies, jobs.data(), k);
        return psa_job_step(jobs[0], k);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PSA_HIP(hipEventCreate(&e0), "hipEventCreate");
    std::unique_ptr<void, void (*)(void *)> g0(e0, [](void *e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); });
    PSA_HIP(hipEventCreate(&e1), "hipEventCreate");
    std::unique_ptr<void, void (*)(void *)> g1(e1, [](void *e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); });
    psa_status st;
    if (warm && (st = advance(warm)) != PSA_OK) return st;
    auto timed = [&](int32_t k, float *ms) -> psa_status {
        PSA_HIP(hipEventRecord(e0, ctx->stream), "hipEventRecord");
        psa_status s2;
        if ((s2 = advance(k)) != PSA_OK) return s2;
        PSA_HIP(hipEventRecord(e1, ctx->stream), "hipEventRecord");
        PSA_HIP(hipEventSynchronize(e1), "hipEventSynchronize");
        PSA_HIP(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime");
        return PSA_OK;
    };
    float t1 = 0.0f, t2 = 0.0f;
    if ((st = timed(probe, &t1)) != PSA_OK) return st;
    double ms = t1;
    if (warm + 3 * probe <= base.steps) {
        if ((st = timed(2 * probe, &t2)) != PSA_OK) return st;
        if (t2 > t1) ms = t2 - t1;
    }
    *us = 1000.0 * ms / probe / copies;
    return PSA_OK;
}

}  // namespace

psa_status tuned_desc(psa_ctx *ctx, const psa_graph *g, psa_run_desc *d, uint32_t mode) {
    d->flags &= ~PSA_TUNE;
    if ((d->flags & PSA_PATH_MASK) != PSA_PATH_AUTO) return PSA_OK;
    psa_tune_result r;
    const psa_status st = psa_tune_get(ctx, g, d, mode, &r);
    if (st != PSA_OK) return st;
    psa_tune_apply(&r, d);
    return PSA_OK;
}

}  // namespace psa

extern "C" {

psa_status psa_autotune(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                        int32_t probe_steps, uint32_t mode, psa_tune_result *out) {
    return psa::guarded("psa_autotune", [&]() -> psa_status {
        if (!ctx || !g || !desc || !out || probe_steps < 1 ||
            (mode != PSA_TUNE_ALONE && mode != PSA_TUNE_BATCH)) {
            psa::set_error("psa_autotune: invalid arguments");
            return PSA_EINVAL;
        }
        if (g->ctx != ctx || desc->steps < 1 || desc->trials < 1) {
            psa::set_error("psa_autotune: graph of another context, or steps / trials < 1");
            return PSA_EINVAL;
        }
        psa_run_desc base = *desc;
        base.flags = PSA_PATH_AUTO;
        const int32_t probe = std::min(probe_steps, base.steps);
        std::vector<psa::Candidate> cands;
        cands.push_back({PSA_PATH_CSR, 4, 0});
        for (int32_t lpt : {1, 2, 4}) {
            // inside a batch a one-trial run uses 2 or 4 lanes per task
            if (mode == PSA_TUNE_BATCH && lpt == 1) continue;
            cands.push_back({PSA_PATH_CSR, 1, lpt});
        }
        const bool dense_ok = psa::dense_encodable(g) && g->info.n <= 32768;
        // the cost models: they also prune the dense candidate of a large
        // graph that they put at more than twice the CSR time (its timing
        // builds an n^2 coupling matrix on the host)
        psa::DevRun mrun;
        mrun.trials = base.trials;
        mrun.t4 = (base.trials + 3) / 4 * 4;
        psa::AnnealPlan mplan;
        std::string why;
        const double model_csr =
            psa::plan_anneal(g->dev, mrun, 0, 0, 0, ctx->max_lds, ctx->num_cu, &mplan, &why)
                ? 1e6 * psa::csr_step_seconds(g->dev, mrun, mplan)
                : -1.0;
        const double model_dense =
            dense_ok ? 1e6 * psa::dense_step_seconds(g->info.n, mrun.t4, psa::dense_two_bit(g), psa::dense_one_bit(g))
                     : -1.0;
        const bool prune_dense = g->info.n > 4096 && model_csr > 0.0 && model_dense > 2.0 * model_csr;
        if (dense_ok && !prune_dense) cands.push_back({PSA_PATH_DENSE, 0, 0});

        psa_tune_result r{};
        r.csr_us_per_step = -1.0;
        r.dense_us_per_step = -1.0;
        r.us_per_step = -1.0;
        for (const psa::Candidate &c : cands) {
            double us = 0.0;
            const psa_status st = psa::time_candidate(ctx, g, base, c, probe, mode, &us);
            if (st == PSA_EUNSUPPORTED) continue;  // e.g. spin state beyond LDS
            if (st != PSA_OK) return st;
            ++r.candidates;
            double &best_of_path = c.path == PSA_PATH_DENSE ? r.dense_us_per_step : r.csr_us_per_step;
            if (best_of_path < 0.0 || us < best_of_path) best_of_path = us;
            if (r.us_per_step < 0.0 || us < r.us_per_step) {
                r.us_per_step = us;
                r.path = c.path;
                r.trials_per_group = c.tpw;
                r.lanes_per_task = c.lpt;
            }
        }
        if (r.candidates == 0) {
            psa::set_error("psa_autotune: no configuration applies to this graph");
            return PSA_EUNSUPPORTED;
        }
        r.model_csr_us = model_csr;
        r.model_dense_us = model_dense;
        {
            std::lock_guard<std::mutex> lock(ctx->tune_mu);
            ctx->tune_cache[psa::tune_key(g, base.trials, mode, base.algorithm)] = r;
        }
        *out = r;
        return PSA_OK;
    });
}

psa_status psa_tune_get(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc, uint32_t mode,
                        psa_tune_result *out) {
    return psa::guarded("psa_tune_get", [&]() -> psa_status {
        if (!ctx || !g || !desc || !out || (mode != PSA_TUNE_ALONE && mode != PSA_TUNE_BATCH) ||
            desc->trials < 1) {
            psa::set_error("psa_tune_get: invalid arguments");
            return PSA_EINVAL;
        }
        {
            std::lock_guard<std::mutex> lock(ctx->tune_mu);
            auto it = ctx->tune_cache.find(psa::tune_key(g, desc->trials, mode, desc->algorithm));
            if (it != ctx->tune_cache.end()) {
                *out = it->second;
                return PSA_OK;
            }
        }
        return psa_autotune(ctx, g, desc, 8, mode, out);
    });
}

void psa_tune_apply(const psa_tune_result *r, psa_run_desc *desc) {
    if (!r || !desc) return;
    desc->flags = (desc->flags & ~(PSA_PATH_MASK | PSA_TUNE)) | r->path;
    desc->trials_per_group = r->trials_per_group;
    desc->lanes_per_task = r->lanes_per_task;
}

int32_t psa_tune_cache_size(psa_ctx *ctx) {
    if (!ctx) return 0;
    try {
        std::lock_guard<std::mutex> lock(ctx->tune_mu);
        return static_cast<int32_t>(ctx->tune_cache.size());
    } catch (...) {
        psa::set_error_static("psa_tune_cache_size: could not lock the tuning cache");
        return -1;
    }
}

void psa_tune_clear(psa_ctx *ctx) {
    if (!ctx) return;
    try {
        std::lock_guard<std::mutex> lock(ctx->tune_mu);
        ctx->tune_cache.clear();
    } catch (...) {
        psa::set_error_static("psa_tune_clear: could not lock the tuning cache");
    }
}

}  // extern "C"
