// abi.cpp -- the extern "C" surface of libpsa (declared in include/psa.h):
// contexts, graph ingestion (edge list or CSR -> validated symmetric CSR on
// the device), runs (jobs) and their read-outs.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "engine.hpp"
#include "psa.h"

namespace psa {

namespace {
thread_local std::string g_last_error;
thread_local const char *g_static_error = nullptr;  // set_error_static's literal
}

void set_error(const std::string &msg) {
    g_static_error = nullptr;
    g_last_error = msg;
}
void set_error_static(const char *msg) noexcept {
    g_last_error.clear();
    g_static_error = msg;
}
void clear_error() {
    g_static_error = nullptr;
    g_last_error.clear();
}
const char *last_error_cstr() { return g_static_error ? g_static_error : g_last_error.c_str(); }

}  // namespace psa

using psa::set_error;

namespace {


// Bump allocator over memory the caller owns (psa_anneal_noalloc's static
// scratch): 256-byte aligned pieces, never freed.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    void *carve(size_t bytes) {
        const size_t at = (used + 255) / 256 * 256;
        if (at > cap || bytes > cap - at) return nullptr;
        used = at + bytes;
        return base + at;
    }
};

// Place count elements on the device (at least one) -- from `arena` when
// given, else a fresh allocation -- copy src into them when given, and add
// the bytes to *acct.
template <typename T>
psa_status dev_upload(T **dst, const T *src, size_t count, const char *what, size_t *acct,
                      Arena *arena = nullptr) {
    *dst = nullptr;
    if (count == 0) count = 1;
    if (arena) {
        *dst = static_cast<T *>(arena->carve(count * sizeof(T)));
        if (!*dst) {
            set_error(std::string(what) + ": the run needs more than the " +
                      std::to_string(PSA_NOALLOC_SCRATCH_BYTES) +
                      " bytes of the static scratch (at least " +
                      std::to_string(arena->used + count * sizeof(T)) + ")");
            return PSA_ENOMEM;
        }
    } else {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), count * sizeof(T));
        if (e != hipSuccess) {
            *dst = nullptr;
            set_error(std::string(what) + ": device allocation failed");
            return PSA_ENOMEM;
        }
    }
    *acct += count * sizeof(T);
    if (src) {
        hipError_t e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return psa::hip_fail(e, what);
    }
    return PSA_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}


void job_free(psa_job *j) {
    if (!j) return;
    if (j->ctx) {
        (void)hipSetDevice(j->ctx->device);
        (void)hipStreamSynchronize(j->ctx->stream);
    }
    if (j->shares) {
        // the run arrays are the source job's
        j->d_i0 = j->d_lambda = j->d_delta = nullptr;
        j->d_thr24 = nullptr;
        j->d_order = j->d_pp = nullptr;
        j->d_prec = nullptr;
        j->d_pcls = nullptr;
        j->d_pcache = nullptr;
    }
    if (j->borrowed) {
        // carved from memory the job does not own: forget, never free
        j->d_i0 = j->d_lambda = j->d_delta = nullptr;
        j->d_thr24 = nullptr;
        j->d_order = j->d_ring = j->d_pp = nullptr;
        j->d_m = j->d_spins = nullptr;
        j->d_xs = nullptr;
        j->d_scratch = nullptr;
        j->d_prec = nullptr;
        j->d_pcls = nullptr;
        j->d_pcache = nullptr;
    }
    dev_free(j->d_i0);
    dev_free(j->d_lambda);
    dev_free(j->d_delta);
    dev_free(j->d_thr24);
    dev_free(j->d_order);
    dev_free(j->d_m);
    dev_free(j->d_spins);
    dev_free(j->d_xs);
    dev_free(j->d_ring);
    dev_free(j->d_pp);
    dev_free(j->d_prec);
    dev_free(j->d_pcls);
    dev_free(j->d_pcache);
    dev_free(j->d_scratch);
    psa_ctx *ctx = j->retained ? j->ctx : nullptr;
    psa_graph *g = j->graph_ref;
    delete j;
    if (g) psa::graph_unref(g);
    if (ctx) psa::ctx_release(ctx);
}

psa_status ensure_scratch(psa_job *j, size_t bytes) {
    if (j->scratch_bytes >= bytes) return PSA_OK;
    if (j->borrowed) {
        set_error("job: read-out staging beyond what was reserved in the static scratch");
        return PSA_EINVAL;
    }
    PSA_HIP(hipStreamSynchronize(j->ctx->stream), "hipStreamSynchronize");
    dev_free(j->d_scratch);
    j->dev_bytes -= j->scratch_bytes;
    j->scratch_bytes = 0;
    if (hipMalloc(&j->d_scratch, bytes) != hipSuccess) {
        j->d_scratch = nullptr;
        set_error("job: scratch allocation failed");
        return PSA_ENOMEM;
    }
    j->scratch_bytes = bytes;
    j->dev_bytes += bytes;
    return PSA_OK;
}

}  // namespace

extern "C" {

const char *psa_version(void) { return "0.1.0 gfx950"; }

const char *psa_last_error(void) { return psa::last_error_cstr(); }

psa_status psa_ctx_create(int32_t device, void *hip_stream, psa_ctx **out) {
    return psa::guarded("psa_ctx_create", [&]() -> psa_status {
        if (!out) {
            set_error("psa_ctx_create: out is NULL");
            return PSA_EINVAL;
        }
        int count = 0;
        PSA_HIP(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (device < 0 || device >= count) {
            set_error("psa_ctx_create: no HIP device " + std::to_string(device));
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(device), "hipSetDevice");
        // the static scratch of psa_anneal_noalloc: its address on this device
        psa_status sst = psa::noalloc_scratch_init(device);
        if (sst != PSA_OK) return sst;
        psa_ctx *c = new psa_ctx();
        // a failure part-way releases the streams and events made so far
        auto init = [&]() -> psa_status {
            c->device = device;
            PSA_HIP(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device),
                    "hipDeviceGetAttribute");
            int lds = 0;
            PSA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device),
                    "hipDeviceGetAttribute");
            c->max_lds = static_cast<size_t>(lds);
            if (hip_stream) {
                c->stream = static_cast<hipStream_t>(hip_stream);
                c->own_stream = false;
            } else {
                PSA_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
                c->own_stream = true;
            }
            PSA_HIP(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking), "hipStreamCreate");
            PSA_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "hipEventCreate");
            PSA_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "hipEventCreate");
            PSA_HIP(hipStreamCreateWithFlags(&c->stream3, hipStreamNonBlocking), "hipStreamCreate");
            PSA_HIP(hipEventCreateWithFlags(&c->ev_fork3, hipEventDisableTiming), "hipEventCreate");
            PSA_HIP(hipEventCreateWithFlags(&c->ev_join3, hipEventDisableTiming), "hipEventCreate");
            return PSA_OK;
        };
        psa_status ist;
        try {
            ist = init();
        } catch (...) {
            psa::ctx_release(c);
            throw;
        }
        if (ist != PSA_OK) {
            psa::ctx_release(c);
            return ist;
        }
        *out = c;
        return PSA_OK;
    });
}

psa_status psa_ctx_synchronize(psa_ctx *ctx) {
    return psa::guarded("psa_ctx_synchronize", [&]() -> psa_status {
        if (!ctx) {
            set_error("psa_ctx_synchronize: ctx is NULL");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

void psa_ctx_destroy(psa_ctx *ctx) {
    if (!ctx) return;
    try {
        psa::ctx_release(ctx);
    } catch (...) {
        psa::set_error_static("psa_ctx_destroy: exception while releasing the context");
    }
}

psa_status psa_ctx_set_timing(psa_ctx *ctx, int32_t on) {
    return psa::guarded("psa_ctx_set_timing", [&]() -> psa_status {
        if (!ctx) {
            set_error("psa_ctx_set_timing: ctx is NULL");
            return PSA_EINVAL;
        }
        ctx->timing = on != 0;
        return PSA_OK;
    });
}

psa_status psa_debug_dense_wait_limit(psa_ctx *ctx, uint32_t max_polls) {
    return psa::guarded("psa_debug_dense_wait_limit", [&]() -> psa_status {
        if (!ctx) {
            set_error("psa_debug_dense_wait_limit: ctx is NULL");
            return PSA_EINVAL;
        }
        ctx->dense_max_polls = max_polls;
        return PSA_OK;
    });
}

psa_status psa_ctx_set_dense_launch(psa_ctx *ctx, int32_t how) {
    return psa::guarded("psa_ctx_set_dense_launch", [&]() -> psa_status {
        if (!ctx || how < PSA_DENSE_LAUNCH_STEPS || how > PSA_DENSE_LAUNCH_PERSISTENT) {
            set_error("psa_ctx_set_dense_launch: ctx NULL or unknown launch mode");
            return PSA_EINVAL;
        }
        ctx->dense_launch = how;
        if (how != PSA_DENSE_LAUNCH_GRAPH && !ctx->dense_graph_cache.empty()) {
            PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
            PSA_HIP(hipStreamSynchronize(ctx->stream2), "hipStreamSynchronize");
            for (const auto &dg : ctx->dense_graph_cache) (void)hipGraphExecDestroy(dg.exec);
            ctx->dense_graph_cache.clear();
        }
        return PSA_OK;
    });
}

psa_status psa_ctx_timing_read(psa_ctx *ctx, psa_timing *out) {
    return psa::guarded("psa_ctx_timing_read", [&]() -> psa_status {
        if (!ctx || !out) {
            set_error("psa_ctx_timing_read: NULL argument");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        for (const auto &sp : ctx->spans) {
            PSA_HIP(hipEventSynchronize(sp.end), "hipEventSynchronize");
            float ms = 0.0f;
            PSA_HIP(hipEventElapsedTime(&ms, sp.begin, sp.end), "hipEventElapsedTime");
            ctx->timed_ms[sp.family] += ms;
            ctx->timed_launches[sp.family] += sp.launches;
            ctx->event_pool.push_back(sp.begin);
            ctx->event_pool.push_back(sp.end);
        }
        ctx->spans.clear();
        out->anneal_ms = ctx->timed_ms[psa::kTimeAnneal];
        out->batch_ms = ctx->timed_ms[psa::kTimeBatch];
        out->dense_ms = ctx->timed_ms[psa::kTimeDense];
        out->anneal_launches = ctx->timed_launches[psa::kTimeAnneal];
        out->batch_launches = ctx->timed_launches[psa::kTimeBatch];
        out->dense_launches = ctx->timed_launches[psa::kTimeDense];
        out->dense_graph_launches = ctx->timed_graph_launches;
        for (int f = 0; f < 3; ++f) {
            ctx->timed_ms[f] = 0.0;
            ctx->timed_launches[f] = 0;
        }
        ctx->timed_graph_launches = 0;
        return PSA_OK;
    });
}

}  // extern "C"

namespace psa {

psa_status time_begin(psa_ctx *ctx, hipStream_t stream, hipEvent_t *ev) {
    *ev = nullptr;
    if (!ctx->timing) return PSA_OK;
    if (ctx->event_pool.empty()) {
        PSA_HIP(hipEventCreate(ev), "hipEventCreate");
    } else {
        *ev = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    }
    PSA_HIP(hipEventRecord(*ev, stream), "hipEventRecord");
    return PSA_OK;
}

psa_status time_end(psa_ctx *ctx, hipStream_t stream, int family, hipEvent_t begin,
                    int64_t launches) {
    if (!begin) return PSA_OK;
    hipEvent_t end = nullptr;
    if (ctx->event_pool.empty()) {
        PSA_HIP(hipEventCreate(&end), "hipEventCreate");
    } else {
        end = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    }
    PSA_HIP(hipEventRecord(end, stream), "hipEventRecord");
    ctx->spans.push_back({family, begin, end, launches});
    return PSA_OK;
}

void ctx_retain(psa_ctx *ctx) { ctx->refs.fetch_add(1); }

void ctx_release(psa_ctx *ctx) {
    if (ctx->refs.fetch_sub(1) != 1) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->stream2) (void)hipStreamSynchronize(ctx->stream2);
    if (ctx->stream3) (void)hipStreamSynchronize(ctx->stream3);
    if (ctx->d_batch_table) (void)hipFree(ctx->d_batch_table);
    if (ctx->d_energy_table) (void)hipFree(ctx->d_energy_table);
    if (ctx->d_batch_work) (void)hipFree(ctx->d_batch_work);
    if (ctx->d_dense_table) (void)hipFree(ctx->d_dense_table);
    if (ctx->d_dense_work) (void)hipFree(ctx->d_dense_work);
    for (const auto &dg : ctx->dense_graph_cache) (void)hipGraphExecDestroy(dg.exec);
    if (ctx->d_dense_sync) (void)hipFree(ctx->d_dense_sync);
    if (ctx->h_dense_err) (void)hipHostFree(ctx->h_dense_err);
    for (const auto &sp : ctx->spans) {
        (void)hipEventDestroy(sp.begin);
        (void)hipEventDestroy(sp.end);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->stream2) (void)hipStreamDestroy(ctx->stream2);
    if (ctx->ev_fork3) (void)hipEventDestroy(ctx->ev_fork3);
    if (ctx->ev_join3) (void)hipEventDestroy(ctx->ev_join3);
    if (ctx->stream3) (void)hipStreamDestroy(ctx->stream3);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // namespace psa

extern "C" {

psa_status psa_graph_from_edges(psa_ctx *ctx, int32_t n, int64_t m, const int32_t *u,
                                const int32_t *v, const int32_t *val, const int32_t *h,
                                uint32_t flags, psa_graph **out) {
    return psa::guarded("psa_graph_from_edges", [&]() -> psa_status {
        if (!ctx || !out) {
            set_error("psa_graph_from_edges: invalid arguments");
            return PSA_EINVAL;
        }
        psa::HostGraph hg;
        psa_status st = psa::host_graph_from_edges(n, m, u, v, val, h, flags, &hg);
        if (st != PSA_OK) return st;
        return psa::upload_graph(ctx, std::move(hg), out);
    });
}

psa_status psa_graph_from_csr(psa_ctx *ctx, int32_t n, const int64_t *row_ptr, const int32_t *col,
                              const int32_t *val, const int32_t *h, uint32_t flags,
                              psa_graph **out) {
    return psa::guarded("psa_graph_from_csr", [&]() -> psa_status {
        if (!ctx || !out) {
            set_error("psa_graph_from_csr: invalid arguments");
            return PSA_EINVAL;
        }
        psa::HostGraph hg;
        psa_status st = psa::host_graph_from_csr(n, row_ptr, col, val, h, flags, &hg);
        if (st != PSA_OK) return st;
        return psa::upload_graph(ctx, std::move(hg), out);
    });
}

psa_status psa_graph_info_get(const psa_graph *g, psa_graph_info *out) {
    return psa::guarded("psa_graph_info_get", [&]() -> psa_status {
        if (!g || !out) {
            set_error("psa_graph_info_get: NULL argument");
            return PSA_EINVAL;
        }
        *out = g->info;
        out->device_bytes = static_cast<int64_t>(g->dev_bytes + g->dense_bytes);
        return PSA_OK;
    });
}

psa_status psa_graph_check_edges(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                                 const int32_t *val, const int32_t *h, uint32_t flags,
                                 psa_graph_info *out) {
    return psa::guarded("psa_graph_check_edges", [&]() -> psa_status {
        if (!out) {
            set_error("psa_graph_check_edges: out is NULL");
            return PSA_EINVAL;
        }
        psa::HostGraph hg;
        const psa_status st = psa::host_graph_from_edges(n, m, u, v, val, h, flags, &hg);
        if (st != PSA_OK) return st;
        *out = hg.info;
        out->device_bytes = 0;
        return PSA_OK;
    });
}

void psa_graph_destroy(psa_graph *g) {
    try {
        psa::graph_unref(g);
    } catch (...) {
        psa::set_error_static("psa_graph_destroy: exception while releasing the graph");
    }
}

psa_status psa_schedule_paper(const psa_graph *g, double *i0_min, double *i0_max) {
    return psa::guarded("psa_schedule_paper", [&]() -> psa_status {
        if (!g || !i0_min || !i0_max) {
            set_error("psa_schedule_paper: NULL argument");
            return PSA_EINVAL;
        }
        if (!(g->info.mean_s > 0.0)) {
            set_error("psa_schedule_paper: mean(s_i) is zero (graph has no couplings)");
            return PSA_EINVAL;
        }
        *i0_min = 0.1 / g->info.mean_s;
        *i0_max = 10.0 / g->info.mean_s;
        return PSA_OK;
    });
}

psa_status psa_schedule_fill(int32_t steps, double i0_min, double i0_max, float *i0_out) {
    return psa::guarded("psa_schedule_fill", [&]() -> psa_status {
        return psa::fill_schedule(steps, i0_min, i0_max, i0_out);
    });
}

psa_status psa_periods_draw(int32_t n, uint64_t seed, double sigma_nu, int32_t t_res,
                            uint32_t *period_out) {
    return psa::guarded("psa_periods_draw", [&]() -> psa_status {
        return psa::draw_periods(n, seed, sigma_nu, t_res, period_out);
    });
}

psa_status psa_variability_draw(int32_t n, uint64_t seed, double sigma_lambda,
                                double sigma_delta, double sigma_nu, double p_mean,
                                float *lambda_out, float *delta_out, uint32_t *thr24_out) {
    return psa::guarded("psa_variability_draw", [&]() -> psa_status {
        return psa::draw_variability(n, seed, sigma_lambda, sigma_delta, sigma_nu, p_mean, lambda_out,
                                     delta_out, thr24_out);
    });
}

void psa_run_desc_default(psa_run_desc *d) {
    if (!d) return;
    memset(d, 0, sizeof(*d));
    d->steps = 1000;
    d->trials = 1;
    d->i0_min = -1.0;
    d->i0_max = -1.0;
    d->p_mean = 1.0;
    d->algorithm = PSA_ALG_PSA;
    d->p_stall = 0.5;
    d->window = 4;
}

}  // extern "C"

namespace {

// Body of psa_job_create: validate, upload the schedule and factors, plan
// the launch, set the initial spins.  Device arrays come from `arena` when
// given (then the job borrows them), else from fresh allocations.
psa_status create_job(const char *who, psa_ctx *ctx, const psa_graph *g,
                      const psa_run_desc *desc, Arena *arena, psa_job **out) {
    if (!ctx || !g || !desc || !out) {
        set_error(std::string(who) + ": NULL argument");
        return PSA_EINVAL;
    }
    if (g->ctx != ctx) {
        set_error(std::string(who) + ": graph belongs to another context");
        return PSA_EINVAL;
    }
    const int32_t n = g->info.n;
    if (desc->steps < 1 || desc->trials < 1 || desc->trials > (1 << 28)) {
        set_error(std::string(who) + ": need steps >= 1 and 1 <= trials <= 2^28");
        return PSA_EINVAL;
    }
    if (desc->block != 0 && desc->block != 256 && desc->block != 512 && desc->block != 1024) {
        set_error(std::string(who) + ": block must be 0, 256, 512 or 1024");
        return PSA_EINVAL;
    }
    if (desc->trials_per_group != 0 && desc->trials_per_group != 1 &&
        desc->trials_per_group != 4) {
        set_error(std::string(who) + ": trials_per_group must be 0, 1 or 4");
        return PSA_EINVAL;
    }
    if (desc->lanes_per_task != 0 && desc->lanes_per_task != 1 && desc->lanes_per_task != 2 &&
        desc->lanes_per_task != 4) {
        set_error(std::string(who) + ": lanes_per_task must be 0, 1, 2 or 4");
        return PSA_EINVAL;
    }
    if ((desc->flags & ~(PSA_PATH_MASK | PSA_TUNE)) != 0 ||
        (desc->flags & PSA_PATH_MASK) == PSA_PATH_MASK) {
        set_error(std::string(who) + ": unknown flags");
        return PSA_EINVAL;
    }
    if (desc->algorithm != PSA_ALG_PSA && desc->algorithm != PSA_ALG_SPSA &&
        desc->algorithm != PSA_ALG_TAPSA) {
        set_error(std::string(who) + ": unknown algorithm");
        return PSA_EINVAL;
    }
    if (desc->algorithm == PSA_ALG_TAPSA && (desc->window < 1 || desc->window > 64)) {
        set_error(std::string(who) + ": window must be in [1, 64]");
        return PSA_EINVAL;
    }
    if (desc->t_res < 0 ||
        (desc->t_res > 0 && static_cast<int64_t>(desc->steps) * desc->t_res >= (int64_t{1} << 22))) {
        set_error(std::string(who) + ": t_res must be >= 0 with steps * t_res < 2^22");
        return PSA_EINVAL;
    }
    if (desc->t_res > 0 && desc->algorithm != PSA_ALG_PSA) {
        set_error(std::string(who) + ": period-mode timing is built for plain pSA only");
        return PSA_EUNSUPPORTED;
    }
    if (desc->algorithm == PSA_ALG_SPSA && !(desc->p_stall >= 0.0 && desc->p_stall <= 1.0)) {
        set_error(std::string(who) + ": p_stall must be in [0, 1]");
        return PSA_EINVAL;
    }
    if ((desc->flags & PSA_TUNE) && arena) {
        set_error(std::string(who) + ": PSA_TUNE times scratch runs, which allocate");
        return PSA_EINVAL;
    }
    if (desc->flags & PSA_TUNE) {
        psa_run_desc tuned = *desc;
        psa_status st = psa::tuned_desc(ctx, g, &tuned, PSA_TUNE_ALONE);
        if (st != PSA_OK) return st;
        return psa_job_create(ctx, g, &tuned, out);
    }
    const int32_t S = desc->steps;
    std::vector<float> i0(static_cast<size_t>(S));
    if (desc->i0) {
        for (int32_t t = 0; t < S; ++t) {
            if (!(std::isfinite(desc->i0[t]))) {
                set_error(std::string(who) + ": non-finite I0");
                return PSA_EINVAL;
            }
            i0[t] = desc->i0[t];
        }
    } else {
        double lo = desc->i0_min, hi = desc->i0_max;
        if (!(lo > 0.0)) {
            psa_status st = psa_schedule_paper(g, &lo, &hi);
            if (st != PSA_OK) return st;
        }
        psa_status st = psa::fill_schedule(S, lo, hi, i0.data());
        if (st != PSA_OK) return st;
    }
    std::vector<float> lam(static_cast<size_t>(n)), dlt(static_cast<size_t>(n));
    std::vector<uint32_t> thr(static_cast<size_t>(n));
    if (!desc->lambda || !desc->delta || !desc->thr24) {
        psa_status st = psa::draw_variability(n, desc->seed, desc->sigma_lambda, desc->sigma_delta,
                                              desc->sigma_nu, desc->p_mean, lam.data(), dlt.data(),
                                              thr.data());
        if (st != PSA_OK) return st;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (desc->lambda) lam[i] = desc->lambda[i];
        if (desc->delta) dlt[i] = desc->delta[i];
        if (desc->thr24) thr[i] = desc->thr24[i];
        if (!std::isfinite(lam[i]) || !std::isfinite(dlt[i]) || thr[i] > psa::kGateOneHost) {
            set_error(std::string(who) + ": lambda/delta must be finite and thr24 <= 2^24");
            return PSA_EINVAL;
        }
    }
    if (desc->t_res > 0) {
        // period mode: the per-p-bit timing array holds integer periods
        if (desc->period) {
            for (int32_t i = 0; i < n; ++i) thr[i] = desc->period[i];
        } else {
            psa_status st = psa::draw_periods(n, desc->seed, desc->sigma_nu, desc->t_res, thr.data());
            if (st != PSA_OK) return st;
        }
        for (int32_t i = 0; i < n; ++i)
            if (thr[i] < 1u) {
                set_error(std::string(who) + ": periods must be >= 1");
                return PSA_EINVAL;
            }
    }
    PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    std::unique_ptr<psa_job, void (*)(psa_job *)> j(new psa_job(), job_free);
    j->borrowed = arena != nullptr;
    j->ctx = ctx;
    psa::ctx_retain(ctx);
    j->retained = true;
    const_cast<psa_graph *>(g)->refs.fetch_add(1);
    j->graph_ref = const_cast<psa_graph *>(g);
    j->g = g;
    j->run.trials = desc->trials;
    j->run.t4 = (desc->trials + 3) / 4 * 4;
    j->run.steps = S;
    psa_status st;
    const int32_t n4 = g->dev.n4;
    // input-stage state first: the launch plan depends on it (LDS windows)
    if (desc->algorithm == PSA_ALG_SPSA) {
        // held inputs: [t4/4][n4][4] floats, formed at step 0 before any read
        const size_t xb = static_cast<size_t>(n4) * static_cast<size_t>(j->run.t4);
        if ((st = dev_upload<float>(&j->d_xs, nullptr, xb, "job held inputs", &j->dev_bytes, arena)) != PSA_OK) return st;
        j->run.xs = j->d_xs;
        j->run.stall24 = static_cast<uint32_t>(std::floor(desc->p_stall * 16777216.0));
    }
    if (desc->algorithm == PSA_ALG_TAPSA) {
        // field windows: [t4/4][n4][window][4] int32, slot t mod window written
        // at step t before any read of it
        const size_t rb = static_cast<size_t>(n4) * static_cast<size_t>(j->run.t4) *
                          static_cast<size_t>(desc->window);
        if ((st = dev_upload<int32_t>(&j->d_ring, nullptr, rb, "job field windows", &j->dev_bytes, arena)) != PSA_OK)
            return st;
        j->run.ring = j->d_ring;
        j->run.alpha = desc->window;
    }
    const uint32_t path = desc->flags & PSA_PATH_MASK;
    if (path != PSA_PATH_DENSE) {
        std::string why;
        if (!psa::plan_anneal(g->dev, j->run, desc->trials_per_group, desc->lanes_per_task,
                              desc->block, ctx->max_lds, ctx->num_cu, &j->plan, &why)) {
            if (path == PSA_PATH_CSR) {
                set_error(std::string(who) + ": " + why);
                return PSA_EUNSUPPORTED;
            }
            j->plan.dense = 1;  // too large for the LDS-resident sweep
        }
    }
    if (path == PSA_PATH_DENSE || (path == PSA_PATH_AUTO && psa::prefer_dense(g, j->run, j->plan)))
        j->plan.dense = 1;
    if (j->plan.dense && arena) {
        set_error("the run needs the dense path, which the static scratch does not hold");
        return PSA_EUNSUPPORTED;
    }
    if (j->plan.dense) {
        psa_status st = psa::ensure_dense_matrix(const_cast<psa_graph *>(g));
        if (st != PSA_OK) return st;
        j->plan.nb = desc->trials >= 64 ? 4 : (desc->trials >= 32 ? 2 : 1);
    }
    j->run.key0 = static_cast<uint32_t>(desc->seed);
    j->run.key1 = static_cast<uint32_t>(desc->seed >> 32);
    j->identity_factors = desc->algorithm == PSA_ALG_PSA && desc->t_res == 0;
    for (int32_t i = 0; i < n && j->identity_factors; ++i)
        j->identity_factors = lam[i] == 1.0f && dlt[i] == 0.0f && thr[i] >= psa::kGateOneHost;
    // per-p-bit arrays padded to n4: padding p-bits never fire
    lam.resize(static_cast<size_t>(n4), 1.0f);
    dlt.resize(static_cast<size_t>(n4), 0.0f);
    thr.resize(static_cast<size_t>(n4), 0u);
    std::vector<int32_t> order;
    psa::task_order(g->dev, g->row_ptr_host, j->plan, &order);
    if ((st = dev_upload(&j->d_i0, i0.data(), i0.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
    if ((st = dev_upload(&j->d_lambda, lam.data(), lam.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
    if ((st = dev_upload(&j->d_delta, dlt.data(), dlt.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
    if ((st = dev_upload(&j->d_thr24, thr.data(), thr.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
    if ((st = dev_upload(&j->d_order, order.data(), order.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
    if (g->dev.ell) {
        // per-p-bit constants of the ELL four-trial sweep, one 16-byte load each
        std::vector<int32_t> pp(4 * static_cast<size_t>(n4));
        for (int32_t i = 0; i < n4; ++i) {
            pp[4 * i] = g->h_host[i] - (g->row_ptr_host[i + 1] - g->row_ptr_host[i]);
            memcpy(&pp[4 * i + 1], &lam[i], 4);
            memcpy(&pp[4 * i + 2], &dlt[i], 4);
            pp[4 * i + 3] = static_cast<int32_t>(thr[i]);
        }
        if ((st = dev_upload(&j->d_pp, pp.data(), pp.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
        j->run.pp = j->d_pp;
    }
    if (desc->t_res > 0 && !j->plan.dense && j->plan.tpw == 1) {
        // period mode, one trial per workgroup: the sweep over period classes
        std::vector<psa::PeriodRec> recs;
        std::vector<psa::PeriodClass> classes;
        std::vector<uint32_t> ecache;
        j->run.t_res = desc->t_res;
        if (psa::plan_period(g->dev, j->run, g->row_ptr_host, g->col_host, g->val_host, g->h_host, lam,
                             dlt, thr, ctx->max_lds,
                             desc->block, &j->pplan, &recs, &classes, &ecache)) {
            if ((st = dev_upload(&j->d_prec, recs.data(), recs.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
            if ((st = dev_upload(&j->d_pcls, classes.data(), classes.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK) return st;
            if (!ecache.empty() &&
                (st = dev_upload(&j->d_pcache, ecache.data(), ecache.size(), "job upload", &j->dev_bytes, arena)) != PSA_OK)
                return st;
        } else {
            j->pplan = psa::PeriodPlan{};
        }
    }
    const size_t spin_bytes = static_cast<size_t>(n) * static_cast<size_t>(j->run.t4);
    if ((st = dev_upload<int8_t>(&j->d_spins, nullptr, spin_bytes, "job spins", &j->dev_bytes, arena)) != PSA_OK) return st;
    if (j->plan.dense) {
        j->tp = (j->run.t4 + 16 * j->plan.nb - 1) / (16 * j->plan.nb) * (16 * j->plan.nb);
        const size_t mb = 2 * static_cast<size_t>(j->tp) * static_cast<size_t>(g->np);
        if ((st = dev_upload<int8_t>(&j->d_m, nullptr, mb, "job dense spins", &j->dev_bytes, arena)) != PSA_OK) return st;
    }
    j->run.t_res = desc->t_res;
    j->run.i0 = j->d_i0;
    j->run.lambda = j->d_lambda;
    j->run.delta = j->d_delta;
    j->run.thr24 = j->d_thr24;
    j->run.spins = j->d_spins;
    if (arena) {
        // read-out staging of the energy reduction, reserved before any launch
        const size_t bytes = 2 * static_cast<size_t>(desc->trials) * sizeof(int64_t) +
                             psa::energy_partial_bytes(n, j->run.t4);
        j->d_scratch = arena->carve(bytes);
        if (!j->d_scratch) {
            set_error("the run needs more than the " + std::to_string(PSA_NOALLOC_SCRATCH_BYTES) +
                      " bytes of the static scratch (at least " + std::to_string(arena->used + bytes) +
                      ")");
            return PSA_ENOMEM;
        }
        j->scratch_bytes = bytes;
        j->dev_bytes += bytes;
    }
    PSA_HIP(psa::launch_init_spins(ctx->stream, n, j->run), "init_spins launch");
    j->t = 0;
    *out = j.release();
    return PSA_OK;
}

}  // namespace

namespace psa {

psa_status clone_job_for_timing(psa_job *src, psa_job **out) {
    psa_ctx *ctx = src->ctx;
    PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    std::unique_ptr<psa_job, void (*)(psa_job *)> j(new psa_job(), job_free);
    j->ctx = ctx;
    ctx_retain(ctx);
    j->retained = true;
    src->graph_ref->refs.fetch_add(1);
    j->graph_ref = src->graph_ref;
    j->g = src->g;
    j->run = src->run;
    j->plan = src->plan;
    j->pplan = src->pplan;
    j->tp = src->tp;
    j->identity_factors = src->identity_factors;
    j->shares = src;
    j->d_i0 = src->d_i0;
    j->d_lambda = src->d_lambda;
    j->d_delta = src->d_delta;
    j->d_thr24 = src->d_thr24;
    j->d_order = src->d_order;
    j->d_pp = src->d_pp;
    j->d_prec = src->d_prec;
    j->d_pcls = src->d_pcls;
    j->d_pcache = src->d_pcache;
    psa_status st;
    const int32_t n = src->g->info.n;
    const size_t spin_bytes = static_cast<size_t>(n) * static_cast<size_t>(j->run.t4);
    if ((st = dev_upload<int8_t>(&j->d_spins, nullptr, spin_bytes, "clone spins", &j->dev_bytes)) != PSA_OK) return st;
    j->run.spins = j->d_spins;
    const size_t n4t4 = static_cast<size_t>(src->g->dev.n4) * static_cast<size_t>(j->run.t4);
    if (src->d_xs) {
        if ((st = dev_upload<float>(&j->d_xs, nullptr, n4t4, "clone held inputs", &j->dev_bytes)) != PSA_OK) return st;
        j->run.xs = j->d_xs;
    }
    if (src->d_ring) {
        if ((st = dev_upload<int32_t>(&j->d_ring, nullptr, n4t4 * static_cast<size_t>(j->run.alpha),
                                      "clone field windows", &j->dev_bytes)) != PSA_OK)
            return st;
        j->run.ring = j->d_ring;
    }
    if (src->d_m) {
        const size_t mb = 2 * static_cast<size_t>(j->tp) * static_cast<size_t>(src->g->np);
        if ((st = dev_upload<int8_t>(&j->d_m, nullptr, mb, "clone dense spins", &j->dev_bytes)) != PSA_OK) return st;
    }
    PSA_HIP(launch_init_spins(ctx->stream, n, j->run), "init_spins launch");
    j->t = 0;
    *out = j.release();
    return PSA_OK;
}

}  // namespace psa

extern "C" {

psa_status psa_job_create(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                          psa_job **out) {
    return psa::guarded("psa_job_create", [&]() -> psa_status {
        return create_job("psa_job_create", ctx, g, desc, nullptr, out);
    });
}

psa_status psa_job_reset(psa_job *job) {
    return psa::guarded("psa_job_reset", [&]() -> psa_status {
        if (!job) {
            set_error("psa_job_reset: job is NULL");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        PSA_HIP(psa::launch_init_spins(job->ctx->stream, job->g->info.n, job->run), "init_spins launch");
        job->t = 0;
        return PSA_OK;
    });
}

psa_status psa_job_step(psa_job *job, int32_t k) {
    return psa::guarded("psa_job_step", [&]() -> psa_status {
        if (!job || k < 0) {
            set_error("psa_job_step: invalid arguments");
            return PSA_EINVAL;
        }
        const int32_t t_end = static_cast<int32_t>(std::min<int64_t>(int64_t{job->t} + k, job->run.steps));
        if (t_end <= job->t) return PSA_OK;
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        if (job->plan.dense) {
            psa_ctx *ctx = job->ctx;
            PSA_HIP(hipEventRecord(ctx->ev_fork, ctx->stream), "hipEventRecord");
            PSA_HIP(hipStreamWaitEvent(ctx->stream2, ctx->ev_fork, 0), "hipStreamWaitEvent");
            psa_job *one[1] = {job};
            psa_status st = psa::dense_step_jobs(ctx, one, 1, k);
            PSA_HIP(hipEventRecord(ctx->ev_join, ctx->stream2), "hipEventRecord");
            PSA_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0), "hipStreamWaitEvent");
            return st;
        }
        hipEvent_t ev = nullptr;
        psa_status st = psa::time_begin(job->ctx, job->ctx->stream, &ev);
        if (st != PSA_OK) return st;
        if (job->pplan.nclass > 0)
            PSA_HIP(psa::launch_period(job->ctx->stream, job->g->dev, job->run, job->pplan, job->d_prec,
                                       job->d_pcls, job->d_pcache, job->t, t_end),
                    "period sweep launch");
        else
            PSA_HIP(psa::launch_anneal(job->ctx->stream, job->g->dev, job->run, job->plan, job->d_order,
                                       job->t, t_end),
                    "anneal launch");
        if ((st = psa::time_end(job->ctx, job->ctx->stream, psa::kTimeAnneal, ev, 1)) != PSA_OK) return st;
        job->t = t_end;
        return PSA_OK;
    });
}

psa_status psa_job_get_info(const psa_job *job, psa_job_info *out) {
    return psa::guarded("psa_job_get_info", [&]() -> psa_status {
        if (!job || !out) {
            set_error("psa_job_get_info: NULL argument");
            return PSA_EINVAL;
        }
        out->path = job->plan.dense ? PSA_PATH_DENSE : PSA_PATH_CSR;
        out->trials_per_group = job->plan.dense ? 0 : job->plan.tpw;
        out->lanes_per_task = job->plan.dense ? 0 : job->plan.lpt;
        out->block = job->plan.dense ? 256 : job->plan.block;
        out->dense_encoding = job->plan.dense ? job->g->dense_enc + 1 : 0;
        out->algorithm = job->run.ring ? PSA_ALG_TAPSA : (job->run.xs ? PSA_ALG_SPSA : PSA_ALG_PSA);
        out->device_bytes = static_cast<int64_t>(job->dev_bytes);
        out->period_classes = job->pplan.nclass;
        out->period_resident = job->pplan.resident_k;
        return PSA_OK;
    });
}

psa_status psa_job_position(const psa_job *job, int32_t *t) {
    return psa::guarded("psa_job_position", [&]() -> psa_status {
        if (!job || !t) {
            set_error("psa_job_position: NULL argument");
            return PSA_EINVAL;
        }
        *t = job->t;
        return PSA_OK;
    });
}

psa_status psa_job_read_spins(psa_job *job, int8_t *out, uint32_t flags) {
    return psa::guarded("psa_job_read_spins", [&]() -> psa_status {
        if (!job || !out || (flags & ~PSA_OUT_DEVICE) != 0) {
            set_error("psa_job_read_spins: invalid arguments");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        const int32_t n = job->g->info.n;
        const size_t bytes = static_cast<size_t>(n) * job->run.trials;
        if (flags & PSA_OUT_DEVICE) {
            PSA_HIP(psa::launch_spins_to_tn(job->ctx->stream, n, job->run, out), "spins read-out");
            return PSA_OK;
        }
        psa_status st = ensure_scratch(job, bytes);
        if (st != PSA_OK) return st;
        int8_t *tmp = static_cast<int8_t *>(job->d_scratch);
        PSA_HIP(psa::launch_spins_to_tn(job->ctx->stream, n, job->run, tmp), "spins read-out");
        PSA_HIP(hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, job->ctx->stream), "copy-out");
        PSA_HIP(hipStreamSynchronize(job->ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

psa_status psa_job_write_spins(psa_job *job, const int8_t *in, int32_t t, uint32_t flags) {
    return psa::guarded("psa_job_write_spins", [&]() -> psa_status {
        if (!job || !in || (flags & ~PSA_OUT_DEVICE) != 0 || t < 0 || t > job->run.steps) {
            set_error("psa_job_write_spins: invalid arguments");
            return PSA_EINVAL;
        }
        if ((job->run.xs != nullptr || job->run.ring != nullptr) && t > 0) {
            set_error("psa_job_write_spins: an SpSA or TApSA job resumes only at step 0 (held inputs "
                      "and field windows are not part of the spins)");
            return PSA_EUNSUPPORTED;
        }
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        const int32_t n = job->g->info.n;
        const size_t bytes = static_cast<size_t>(n) * job->run.trials;
        std::vector<int8_t> host(bytes);
        if (flags & PSA_OUT_DEVICE) {
            PSA_HIP(hipStreamSynchronize(job->ctx->stream), "hipStreamSynchronize");
            PSA_HIP(hipMemcpy(host.data(), in, bytes, hipMemcpyDeviceToHost), "copy-in");
        } else {
            memcpy(host.data(), in, bytes);
        }
        for (size_t p = 0; p < bytes; ++p)
            if (host[p] != 1 && host[p] != -1) {
                set_error("psa_job_write_spins: spins must be +1 or -1");
                return PSA_EINVAL;
            }
        psa_status st = ensure_scratch(job, bytes);
        if (st != PSA_OK) return st;
        int8_t *tmp = static_cast<int8_t *>(job->d_scratch);
        PSA_HIP(hipMemcpyAsync(tmp, host.data(), bytes, hipMemcpyHostToDevice, job->ctx->stream),
                "copy-in");
        PSA_HIP(psa::launch_spins_from_tn(job->ctx->stream, n, job->run, tmp), "spins write");
        PSA_HIP(hipStreamSynchronize(job->ctx->stream), "hipStreamSynchronize");
        job->t = t;
        return PSA_OK;
    });
}

psa_status psa_job_local_field(psa_job *job, int32_t *out, uint32_t flags) {
    return psa::guarded("psa_job_local_field", [&]() -> psa_status {
        if (!job || !out || (flags & ~PSA_OUT_DEVICE) != 0) {
            set_error("psa_job_local_field: invalid arguments");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        const int32_t n = job->g->info.n;
        const size_t bytes = static_cast<size_t>(n) * job->run.trials * sizeof(int32_t);
        if (flags & PSA_OUT_DEVICE) {
            PSA_HIP(psa::launch_local_field(job->ctx->stream, job->g->dev, job->run, out), "local field");
            return PSA_OK;
        }
        psa_status st = ensure_scratch(job, bytes);
        if (st != PSA_OK) return st;
        int32_t *tmp = static_cast<int32_t *>(job->d_scratch);
        PSA_HIP(psa::launch_local_field(job->ctx->stream, job->g->dev, job->run, tmp), "local field");
        PSA_HIP(hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, job->ctx->stream), "copy-out");
        PSA_HIP(hipStreamSynchronize(job->ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

psa_status psa_job_energy_cut(psa_job *job, int64_t *energy, int64_t *cut, uint32_t flags) {
    return psa::guarded("psa_job_energy_cut", [&]() -> psa_status {
        if (!job || !energy || !cut || (flags & ~PSA_OUT_DEVICE) != 0) {
            set_error("psa_job_energy_cut: invalid arguments");
            return PSA_EINVAL;
        }
        PSA_HIP(hipSetDevice(job->ctx->device), "hipSetDevice");
        // scratch: [energy, cut staging (host outputs)][per-block partial sums]
        const size_t bytes = static_cast<size_t>(job->run.trials) * sizeof(int64_t);
        const size_t part_bytes = psa::energy_partial_bytes(job->g->info.n, job->run.t4);
        psa_status st = ensure_scratch(job, 2 * bytes + part_bytes);
        if (st != PSA_OK) return st;
        int64_t *tmp = static_cast<int64_t *>(job->d_scratch);
        int64_t *part = tmp + 2 * job->run.trials;
        if (flags & PSA_OUT_DEVICE) {
            PSA_HIP(psa::launch_energy_cut(job->ctx->stream, job->g->dev, job->run, part, energy, cut),
                    "energy/cut");
            return PSA_OK;
        }
        PSA_HIP(psa::launch_energy_cut(job->ctx->stream, job->g->dev, job->run, part, tmp,
                                       tmp + job->run.trials),
                "energy/cut");
        PSA_HIP(hipMemcpyAsync(energy, tmp, bytes, hipMemcpyDeviceToHost, job->ctx->stream), "copy-out");
        PSA_HIP(hipMemcpyAsync(cut, tmp + job->run.trials, bytes, hipMemcpyDeviceToHost,
                               job->ctx->stream),
                "copy-out");
        PSA_HIP(hipStreamSynchronize(job->ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

psa_status psa_jobs_energy_cut(psa_ctx *ctx, int32_t count, psa_job *const *jobs, int64_t *const *energy,
                               int64_t *const *cut, uint32_t flags) {
    return psa::guarded("psa_jobs_energy_cut", [&]() -> psa_status {
        if (!ctx || count < 0 || (count > 0 && (!jobs || !energy || !cut)) || (flags & ~PSA_OUT_DEVICE) != 0) {
            set_error("psa_jobs_energy_cut: invalid arguments");
            return PSA_EINVAL;
        }
        for (int32_t j = 0; j < count; ++j)
            if (!jobs[j] || jobs[j]->ctx != ctx || !energy[j] || !cut[j]) {
                set_error("psa_jobs_energy_cut: job " + std::to_string(j) +
                          " is NULL, belongs to another context, or has no outputs");
                return PSA_EINVAL;
            }
        if (count == 0) return PSA_OK;
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        const bool device = (flags & PSA_OUT_DEVICE) != 0;
        std::vector<psa::EnergyJob> table(static_cast<size_t>(count));
        int64_t wgs = 0, trials = 0;
        for (int32_t j = 0; j < count; ++j) {
            psa_job *job = jobs[j];
            // each run's partial sums (and host staging) in its own scratch,
            // laid out as psa_job_energy_cut lays them out
            const size_t bytes = static_cast<size_t>(job->run.trials) * sizeof(int64_t);
            const psa_status st =
                ensure_scratch(job, 2 * bytes + psa::energy_partial_bytes(job->g->info.n, job->run.t4));
            if (st != PSA_OK) return st;
            int64_t *tmp = static_cast<int64_t *>(job->d_scratch);
            psa::EnergyJob &e = table[static_cast<size_t>(j)];
            e.n = job->g->info.n;
            e.t4 = job->run.t4;
            e.trials = job->run.trials;
            e.blocks = (e.n + 255) / 256;
            // rows of mean degree 48 or more are read by 16 lanes, of 12 or
            // more by 4 (contiguous column reads), sparser rows by one lane
            const int64_t deg = e.n > 0 ? job->g->dev.nnz / e.n : 0;
            e.lpr = deg >= 48 ? 16 : deg >= 12 ? 4 : 1;
            e.wg0 = static_cast<int32_t>(wgs);
            e.k0 = static_cast<int32_t>(trials);
            e.w2 = job->g->dev.w2;
            e.row_ptr = job->g->dev.row_ptr;
            e.col = job->g->dev.col;
            e.val = job->g->dev.val;
            e.h = job->g->dev.h;
            e.spins = job->run.spins;
            e.part = tmp + 2 * job->run.trials;
            e.energy = device ? energy[j] : tmp;
            e.cut = device ? cut[j] : tmp + job->run.trials;
            wgs += psa::energy_batch_wgs(e.n, e.t4);
            trials += e.trials;
            if (wgs > std::numeric_limits<int32_t>::max() || trials > std::numeric_limits<int32_t>::max()) {
                set_error("psa_jobs_energy_cut: too many runs for one read-out");
                return PSA_EINVAL;
            }
        }
        // the table buffer is reused: the previous read-out must be done
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        const size_t tbytes = table.size() * sizeof(psa::EnergyJob);
        if (ctx->energy_table_cap < tbytes) {
            if (ctx->d_energy_table) (void)hipFree(ctx->d_energy_table);
            ctx->d_energy_table = nullptr;
            ctx->energy_table_cap = 0;
            if (hipMalloc(&ctx->d_energy_table, tbytes) != hipSuccess) {
                ctx->d_energy_table = nullptr;
                set_error("psa_jobs_energy_cut: device allocation failed");
                return PSA_ENOMEM;
            }
            ctx->energy_table_cap = tbytes;
        }
        ctx->h_energy_table = std::move(table);
        PSA_HIP(hipMemcpyAsync(ctx->d_energy_table, ctx->h_energy_table.data(), tbytes, hipMemcpyHostToDevice,
                               ctx->stream),
                "energy table upload");
        PSA_HIP(psa::launch_energy_cut_batch(ctx->stream, static_cast<const psa::EnergyJob *>(ctx->d_energy_table),
                                             count, static_cast<int32_t>(wgs), static_cast<int32_t>(trials)),
                "energy/cut");
        if (device) return PSA_OK;
        for (int32_t j = 0; j < count; ++j) {
            const psa::EnergyJob &e = ctx->h_energy_table[static_cast<size_t>(j)];
            const size_t bytes = static_cast<size_t>(e.trials) * sizeof(int64_t);
            PSA_HIP(hipMemcpyAsync(energy[j], e.energy, bytes, hipMemcpyDeviceToHost, ctx->stream), "copy-out");
            PSA_HIP(hipMemcpyAsync(cut[j], e.cut, bytes, hipMemcpyDeviceToHost, ctx->stream), "copy-out");
        }
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

void psa_job_destroy(psa_job *job) {
    try {
        job_free(job);
    } catch (...) {
        psa::set_error_static("psa_job_destroy: exception while releasing the job");
    }
}

psa_status psa_anneal(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                      int8_t *spins_out, int64_t *energy_out, int64_t *cut_out, uint32_t flags) {
    return psa::guarded("psa_anneal", [&]() -> psa_status {
        if (!energy_out || !cut_out || (flags & ~PSA_OUT_DEVICE) != 0) {
            set_error("psa_anneal: energy_out and cut_out are required");
            return PSA_EINVAL;
        }
        psa_job *job = nullptr;
        psa_status st = psa_job_create(ctx, g, desc, &job);
        if (st != PSA_OK) return st;
        std::unique_ptr<psa_job, void (*)(psa_job *)> guard(job, job_free);
        if ((st = psa_job_step(job, desc->steps)) != PSA_OK) return st;
        if ((st = psa_job_energy_cut(job, energy_out, cut_out, flags)) != PSA_OK) return st;
        if (spins_out && (st = psa_job_read_spins(job, spins_out, flags)) != PSA_OK) return st;
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

psa_status psa_anneal_noalloc(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                              int8_t *spins_out, int64_t *energy_out, int64_t *cut_out) {
    return psa::guarded("psa_anneal_noalloc", [&]() -> psa_status {
        if (!ctx || !g || !desc || !energy_out || !cut_out) {
            set_error("psa_anneal_noalloc: ctx, g, desc, energy_out and cut_out are required");
            return PSA_EINVAL;
        }
        const uint32_t path = desc->flags & PSA_PATH_MASK;
        if (path == PSA_PATH_DENSE) {
            set_error("psa_anneal_noalloc: the dense path builds its coupling matrix on the device; "
                      "use psa_anneal");
            return PSA_EUNSUPPORTED;
        }
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        void *base = psa::noalloc_scratch(ctx->device);
        if (!base) {
            set_error("psa_anneal_noalloc: no static scratch on this device");
            return PSA_EHIP;
        }
        // earlier work of this context may still read the scratch
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        psa_run_desc d = *desc;
        if (path == PSA_PATH_AUTO) d.flags = (d.flags & ~PSA_PATH_MASK) | PSA_PATH_CSR;
        Arena arena;
        arena.base = static_cast<char *>(base);
        arena.cap = PSA_NOALLOC_SCRATCH_BYTES;
        psa_job *job = nullptr;
        psa_status st = create_job("psa_anneal_noalloc", ctx, g, &d, &arena, &job);
        if (st != PSA_OK) return st;
        std::unique_ptr<psa_job, void (*)(psa_job *)> guard(job, job_free);
        if ((st = psa_job_step(job, d.steps)) != PSA_OK) return st;
        if ((st = psa_job_energy_cut(job, energy_out, cut_out, PSA_OUT_DEVICE)) != PSA_OK) return st;
        if (spins_out && (st = psa_job_read_spins(job, spins_out, PSA_OUT_DEVICE)) != PSA_OK)
            return st;
        PSA_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return PSA_OK;
    });
}

psa_status psa_debug_tanh(psa_ctx *ctx, int64_t count, const float *x, float *y) {
    return psa::guarded("psa_debug_tanh", [&]() -> psa_status {
        if (!ctx || count < 0 || (count > 0 && (!x || !y))) {
            set_error("psa_debug_tanh: invalid arguments");
            return PSA_EINVAL;
        }
        if (count == 0) return PSA_OK;
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        PSA_HIP(psa::launch_debug_tanh(ctx->stream, count, x, y), "debug_tanh launch");
        return PSA_OK;
    });
}

psa_status psa_debug_decide(psa_ctx *ctx, int64_t count, const float *x, const uint32_t *rword,
                            uint8_t *out) {
    return psa::guarded("psa_debug_decide", [&]() -> psa_status {
        if (!ctx || count < 0 || (count > 0 && (!x || !rword || !out))) {
            set_error("psa_debug_decide: invalid arguments");
            return PSA_EINVAL;
        }
        if (count == 0) return PSA_OK;
        PSA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        PSA_HIP(psa::launch_debug_decide(ctx->stream, count, x, rword, out), "debug_decide launch");
        return PSA_OK;
    });
}

}  // extern "C"
