// server.cpp -- serving loop with continuous batching.
//
// A scheduler thread owns the device work of the server's context.  Clients
// submit anneal jobs (edge list + run description + output buffers) from any
// thread.  Between step quanta the scheduler
//   1. retires jobs that reached the end of their schedule (energy, cut and
//      optional spins into the client's buffers, device memory released),
//   2. admits waiting jobs first-come first-served while their HBM footprint
//      fits the budget and a resident slot is free (graph upload, job
//      creation and initial spins happen here; the CPU part of ingestion --
//      validation, CSR, packed encodings -- has already been done by a pool
//      of preparation threads, so it never stalls the device),
//   3. advances every resident job by one quantum of steps with a single
//      batched launch, so requests that arrive while others run join the
//      next launch.
// Results are identical to running each job alone: every random word is
// addressed by (seed, step, p-bit, trial) and each job's spins and step
// counter stay resident between quanta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.hpp"
#include "psa.h"

using psa::set_error;

namespace {

using Clock = std::chrono::steady_clock;

struct ServerJob {
    uint64_t ticket = 0;
    // request (host copies)
    int32_t n = 0;
    std::vector<int32_t> u, v, val, h;
    uint32_t graph_flags = 0;
    psa_run_desc desc{};
    std::vector<float> i0, lambda, delta;
    std::vector<uint32_t> thr24;
    int64_t *energy_out = nullptr;
    int64_t *cut_out = nullptr;
    int8_t *spins_out = nullptr;
    psa::HostGraph hg;     // filled by a preparation thread
    bool prepared = false;
    // state
    int32_t status = PSA_JOB_QUEUED;
    int32_t error = PSA_OK;
    std::string message;
    bool cancel = false;
    size_t footprint = 0;  // device bytes counted against the budget
    psa_graph *graph = nullptr;
    psa_job *job = nullptr;
    int64_t submit_us = 0, admit_us = -1, start_us = -1, end_us = -1;
};

// Device bytes of the read-out at the end of a job (energy / cut staging and
// the reduction's partial sums; the spins when the client asked for them).
size_t readout_bytes(int32_t n, int32_t trials, bool spins) {
    const size_t t4 = static_cast<size_t>((trials + 3) / 4 * 4);
    const size_t ec = 2 * static_cast<size_t>(trials) * sizeof(int64_t) +
                      psa::energy_partial_bytes(n, static_cast<int32_t>(t4));
    return std::max(ec, spins ? static_cast<size_t>(n) * static_cast<size_t>(trials) : size_t{0});
}

// Upper bound of the device bytes a prepared job will hold while resident,
// reserved at admission: the graph in the encodings built for it, the dense
// coupling matrix and dense spin buffers when the dense path may be chosen,
// the run state (schedule, factors, task order, spins, input-stage state,
// per-p-bit constants), the read-out, and -- with PSA_TUNE -- the scratch
// runs the autotuner times (at most 16 copies of the run state).
size_t reserve_of(const psa::HostGraph &hg, const psa_run_desc &d, bool spins) {
    const size_t n = static_cast<size_t>(hg.n);
    const size_t n4 = static_cast<size_t>(hg.n4);
    const size_t t4 = static_cast<size_t>((d.trials + 3) / 4 * 4);
    auto bytes = [](const auto &v) { return v.size() * sizeof(v[0]); };
    const size_t graph = bytes(hg.rp32) + bytes(hg.col) + bytes(hg.val) + bytes(hg.h) +
                         bytes(hg.pk32) + bytes(hg.pk16) + bytes(hg.ux16) + bytes(hg.ell) +
                         bytes(hg.eptr);
    const size_t window = d.algorithm == PSA_ALG_TAPSA ? static_cast<size_t>(std::max(d.window, 1)) : 0;
    size_t run = static_cast<size_t>(d.steps) * 4 + 3 * n4 * 4 + n4 + n * t4 + 16 * n4 +
                 (d.algorithm == PSA_ALG_SPSA ? n4 * t4 * 4 : 0) + n4 * t4 * 4 * window;
    const uint32_t path = d.flags & PSA_PATH_MASK;
    bool encodable = hg.n <= 32768;
    bool one_mag = true;
    int32_t mag = 0;
    for (int32_t v : hg.val) {
        const int32_t a = v < 0 ? -v : v;
        if (a > 127) encodable = false;
        if (mag == 0) mag = a;
        one_mag = one_mag && a == mag;
    }
    encodable = encodable || (one_mag && hg.n <= 32768);
    size_t dense = 0;
    if (path != PSA_PATH_CSR && encodable) {
        const size_t np = static_cast<size_t>(one_mag ? (hg.n + 255) / 256 * 256 : (hg.n + 127) / 128 * 128);
        dense = one_mag ? np * np / 4 : np * np;
        run += 2 * ((t4 + 63) / 64 * 64) * np;
    }
    const bool tune = (d.flags & PSA_TUNE) && path == PSA_PATH_AUTO;
    return graph + dense + run * (tune ? 17 : 1) + readout_bytes(hg.n, d.trials, spins) +
           32 * 256;  // allocation granularity slack
}

// Device bytes a created job holds, its graph's included, plus what its
// read-out will add.
size_t held_bytes(psa_graph *g, psa_job *job, int32_t n, int32_t trials, bool spins) {
    psa_graph_info gi{};
    psa_job_info ji{};
    (void)psa_graph_info_get(g, &gi);
    (void)psa_job_get_info(job, &ji);
    return static_cast<size_t>(gi.device_bytes) + static_cast<size_t>(ji.device_bytes) +
           readout_bytes(n, trials, spins);
}

}  // namespace

struct psa_server {
    psa_ctx *ctx = nullptr;
    psa_server_opts opts{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;  // submissions, cancels, shutdown
    std::condition_variable cv_done;  // job completions
    std::condition_variable cv_prep;  // jobs to prepare
    std::deque<ServerJob *> to_prepare;
    std::vector<std::thread> preparers;
    std::deque<ServerJob *> waiting;  // submit order; admitted once prepared
    std::vector<ServerJob *> resident;
    std::unordered_map<uint64_t, std::unique_ptr<ServerJob>> jobs;
    uint64_t next_ticket = 1;
    size_t used_bytes = 0, peak_used = 0;
    int32_t peak_resident = 0;
    int64_t completed = 0, failed = 0, canceled = 0, quanta = 0;
    bool stop = false;
    std::thread worker;

    int64_t now_us() const {
        return std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0).count();
    }
};

namespace {

void release_device(ServerJob *j) {
    if (j->job) psa_job_destroy(j->job);
    if (j->graph) psa_graph_destroy(j->graph);
    j->job = nullptr;
    j->graph = nullptr;
}

// CPU part of graph ingestion, on a preparation thread.
void preparer(psa_server *s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_prep.wait(lk, [s] { return s->stop || !s->to_prepare.empty(); });
        if (s->to_prepare.empty()) return;  // stopping
        ServerJob *j = s->to_prepare.front();
        s->to_prepare.pop_front();
        lk.unlock();
        psa::HostGraph hg;
        size_t reserve = 0;
        std::string msg;
        const psa_status st = psa::guarded("server: graph preparation", [&]() -> psa_status {
            const psa_status r = psa::host_graph_from_edges(
                j->n, static_cast<int64_t>(j->u.size()), j->u.data(), j->v.data(), j->val.data(),
                j->h.empty() ? nullptr : j->h.data(), j->graph_flags, &hg);
            if (r == PSA_OK) reserve = reserve_of(hg, j->desc, j->spins_out != nullptr);
            return r;
        });
        if (st != PSA_OK) msg = psa_last_error();
        lk.lock();
        j->prepared = true;
        if (st == PSA_OK) {
            j->hg = std::move(hg);
            j->footprint = reserve;
        } else {
            j->error = st;
            j->message = std::move(msg);
        }
        s->cv_work.notify_one();
    }
}

// Upload the graph and create the job on the device (called without the lock).
psa_status admit_job(psa_server *s, ServerJob *j) {
    psa_status st = psa::upload_graph(s->ctx, std::move(j->hg), &j->graph);
    if (st != PSA_OK) return st;
    psa_run_desc d = j->desc;
    d.i0 = j->i0.empty() ? nullptr : j->i0.data();
    d.lambda = j->lambda.empty() ? nullptr : j->lambda.data();
    d.delta = j->delta.empty() ? nullptr : j->delta.data();
    d.thr24 = j->thr24.empty() ? nullptr : j->thr24.data();
    if (d.flags & PSA_TUNE) {
        st = psa::tuned_desc(s->ctx, j->graph, &d, PSA_TUNE_BATCH);
        if (st != PSA_OK) return st;
    }
    if (d.trials_per_group == 0) d.trials_per_group = 1;
    st = psa_job_create(s->ctx, j->graph, &d, &j->job);
    if (st != PSA_OK) return st;
    // the autotuner may have built the dense matrix for a run that reads the CSR
    psa_job_info ji{};
    if ((st = psa_job_get_info(j->job, &ji)) != PSA_OK) return st;
    if (ji.path != PSA_PATH_DENSE) psa::release_dense_matrix(j->graph);
    return PSA_OK;
}

// Energies and cuts of the jobs that finished in one quantum into the
// clients' buffers, in one batched read-out (called without the lock).
psa_status finish_jobs(psa_server *s, const std::vector<ServerJob *> &done) {
    std::vector<psa_job *> jobs;
    std::vector<int64_t *> energy, cut;
    for (ServerJob *j : done) {
        jobs.push_back(j->job);
        energy.push_back(j->energy_out);
        cut.push_back(j->cut_out);
    }
    return psa_jobs_energy_cut(s->ctx, static_cast<int32_t>(jobs.size()), jobs.data(), energy.data(), cut.data(),
                               PSA_OUT_HOST);
}

void scheduler_loop(psa_server *s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // drop prepared jobs that were canceled or failed preparation
        for (auto it = s->waiting.begin(); it != s->waiting.end();) {
            ServerJob *j = *it;
            if (j->prepared && (j->cancel || j->error != PSA_OK)) {
                if (j->cancel) {
                    j->status = PSA_JOB_CANCELED;
                    ++s->canceled;
                } else {
                    j->status = PSA_JOB_ERROR;
                    ++s->failed;
                }
                j->end_us = s->now_us();
                it = s->waiting.erase(it);
                s->cv_done.notify_all();
            } else {
                ++it;
            }
        }
        // admission: first come first served among prepared jobs, by
        // footprint and slot cap (called with the lock held; drops it while
        // a job is uploaded and created)
        auto admit_waiting = [&]() {
            while (!s->stop && static_cast<int32_t>(s->resident.size()) < s->opts.max_resident) {
                auto it = std::find_if(s->waiting.begin(), s->waiting.end(),
                                       [](const ServerJob *x) { return x->prepared; });
                if (it == s->waiting.end()) break;
                ServerJob *j = *it;
                if (s->used_bytes + j->footprint > static_cast<size_t>(s->opts.hbm_budget_bytes)) {
                    if (!s->resident.empty()) break;  // wait for memory to free up
                    // alone it cannot fit: reject
                    s->waiting.erase(it);
                    j->status = PSA_JOB_ERROR;
                    j->error = PSA_ENOMEM;
                    j->message = "job footprint exceeds the server's HBM budget";
                    j->end_us = s->now_us();
                    ++s->failed;
                    s->cv_done.notify_all();
                    continue;
                }
                s->waiting.erase(it);
                s->used_bytes += j->footprint;
                j->admit_us = s->now_us();
                lk.unlock();
                const psa_status st =
                    psa::guarded("server: admission", [&]() -> psa_status { return admit_job(s, j); });
                std::string msg = st == PSA_OK ? "" : psa_last_error();
                // the reservation becomes the bytes the job actually holds
                const size_t held =
                    st == PSA_OK ? held_bytes(j->graph, j->job, j->n, j->desc.trials, j->spins_out != nullptr)
                                 : 0;
                lk.lock();
                if (st != PSA_OK) {
                    release_device(j);
                    s->used_bytes -= j->footprint;
                    j->status = PSA_JOB_ERROR;
                    j->error = st;
                    j->message = msg;
                    j->end_us = s->now_us();
                    ++s->failed;
                    s->cv_done.notify_all();
                    continue;
                }
                s->used_bytes = s->used_bytes - j->footprint + held;
                j->footprint = held;
                j->status = PSA_JOB_RUNNING;
                s->resident.push_back(j);
                s->peak_resident = std::max(s->peak_resident, static_cast<int32_t>(s->resident.size()));
                s->peak_used = std::max(s->peak_used, s->used_bytes);
            }
        };
        if (s->resident.empty()) {
            admit_waiting();
        }
        if (s->resident.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk, [s] {
                if (s->stop) return true;
                for (const ServerJob *x : s->waiting)
                    if (x->prepared) return true;
                return false;
            });
            continue;
        }
        // one quantum over every resident job
        std::vector<ServerJob *> batch = s->resident;
        std::vector<psa_job *> handles;
        const int64_t launch_us = s->now_us();
        for (ServerJob *j : batch) {
            handles.push_back(j->job);
            if (j->start_us < 0) j->start_us = launch_us;
        }
        const int32_t quantum = s->opts.quantum_steps;
        lk.unlock();
        psa_status st = psa_jobs_step_batch(s->ctx, static_cast<int32_t>(handles.size()),
                                            handles.data(), quantum);
        // while the quantum runs: admit waiting jobs (graph upload, job
        // creation, tuning probes queued behind the quantum); they join the
        // next quantum
        lk.lock();
        admit_waiting();
        lk.unlock();
        if (st == PSA_OK) st = psa_ctx_synchronize(s->ctx);
        std::string qmsg = st == PSA_OK ? "" : psa_last_error();
        // retire finished (or failed / canceled) jobs
        std::vector<std::pair<ServerJob *, psa_status>> retired;
        std::vector<ServerJob *> finished;
        for (ServerJob *j : batch) {
            int32_t t = 0;
            psa_job_position(j->job, &t);
            bool cancel;
            {
                std::lock_guard<std::mutex> g(s->mu);
                cancel = j->cancel;
            }
            if (st != PSA_OK) {
                retired.emplace_back(j, st);
            } else if (cancel) {
                retired.emplace_back(j, PSA_ECANCELED);
            } else if (t >= j->desc.steps) {
                finished.push_back(j);
            }
        }
        if (!finished.empty()) {
            const psa_status fs = finish_jobs(s, finished);
            if (fs != PSA_OK) qmsg = psa_last_error();
            for (ServerJob *j : finished) {
                psa_status js = fs;
                if (js == PSA_OK && j->spins_out &&
                    (js = psa_job_read_spins(j->job, j->spins_out, PSA_OUT_HOST)) != PSA_OK)
                    qmsg = psa_last_error();
                retired.emplace_back(j, js);
            }
        }
        for (auto &r : retired) release_device(r.first);
        lk.lock();
        ++s->quanta;
        for (auto &r : retired) {
            ServerJob *j = r.first;
            s->resident.erase(std::find(s->resident.begin(), s->resident.end(), j));
            s->used_bytes -= j->footprint;
            j->end_us = s->now_us();
            if (r.second == PSA_OK) {
                j->status = PSA_JOB_DONE;
                ++s->completed;
            } else if (r.second == PSA_ECANCELED) {
                j->status = PSA_JOB_CANCELED;
                ++s->canceled;
            } else {
                j->status = PSA_JOB_ERROR;
                j->error = r.second;
                j->message = qmsg;
                ++s->failed;
            }
        }
        if (!retired.empty()) s->cv_done.notify_all();
        if (s->stop && s->waiting.empty() && s->resident.empty()) break;
    }
    // shutdown: whatever is still queued is canceled
    for (ServerJob *j : s->waiting) {
        j->status = PSA_JOB_CANCELED;
        j->end_us = s->now_us();
        ++s->canceled;
    }
    s->waiting.clear();
    s->cv_done.notify_all();
}

// The scheduler thread.  Should its loop throw (a failed host allocation),
// every job it holds ends in ERROR and the server stops taking work, instead
// of the exception ending the process.
void scheduler(psa_server *s) {
    psa_status st = PSA_EINTERNAL;
    try {
        scheduler_loop(s);
        return;
    } catch (const std::bad_alloc &) {
        st = PSA_ENOMEM;
    } catch (...) {
    }
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    const int64_t now = s->now_us();
    // resident jobs keep their device memory until psa_server_destroy
    auto fail = [&](ServerJob *j) {
        j->status = PSA_JOB_ERROR;
        j->error = st;
        try {
            j->message = "the server's scheduler stopped on an internal failure";
        } catch (...) {
        }
        j->end_us = now;
        ++s->failed;
    };
    for (ServerJob *j : s->waiting) fail(j);
    for (ServerJob *j : s->resident) fail(j);
    s->waiting.clear();
    s->cv_done.notify_all();
    s->cv_prep.notify_all();
}

void fill_result(const ServerJob *j, psa_result *out) {
    out->status = j->status;
    out->error = j->error;
    out->submit_us = j->submit_us;
    out->admit_us = j->admit_us;
    out->start_us = j->start_us;
    out->end_us = j->end_us;
}

}  // namespace

namespace psa {
void server_shutdown(psa_server *s);
}

extern "C" {

psa_status psa_server_create(psa_ctx *ctx, const psa_server_opts *opts, psa_server **out) {
    return psa::guarded("psa_server_create", [&]() -> psa_status {
        if (!ctx || !out) {
            set_error("psa_server_create: NULL argument");
            return PSA_EINVAL;
        }
        psa_server_opts o{};
        if (opts) o = *opts;
        if (o.hbm_budget_bytes <= 0) {
            size_t free_b = 0, total_b = 0;
            (void)hipSetDevice(ctx->device);
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = size_t{1} << 32;
            o.hbm_budget_bytes = static_cast<int64_t>(free_b / 2);
        }
        if (o.max_resident <= 0) o.max_resident = 64;
        if (o.quantum_steps <= 0) o.quantum_steps = 250;
        if (o.max_waiting < 0) o.max_waiting = 0;
        std::unique_ptr<psa_server> s(new psa_server());
        s->ctx = ctx;
        s->opts = o;
        s->t0 = Clock::now();
        try {
            s->worker = std::thread(scheduler, s.get());
            const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
            for (unsigned k = 0; k < std::min(8u, hw / 2); ++k)
                s->preparers.emplace_back(preparer, s.get());
        } catch (...) {
            // stop and join what was started before the failure, then report it
            {
                std::lock_guard<std::mutex> g(s->mu);
                s->stop = true;
                s->cv_work.notify_all();
                s->cv_prep.notify_all();
            }
            for (std::thread &t : s->preparers)
                if (t.joinable()) t.join();
            if (s->worker.joinable()) s->worker.join();
            throw;
        }
        *out = s.release();
        return PSA_OK;
    });
}

psa_status psa_server_submit(psa_server *s, int32_t n, int64_t m, const int32_t *u,
                             const int32_t *v, const int32_t *val, const int32_t *h,
                             uint32_t graph_flags, const psa_run_desc *desc, int64_t *energy_out,
                             int64_t *cut_out, int8_t *spins_out, uint64_t *ticket) {
    return psa::guarded("psa_server_submit", [&]() -> psa_status {
        if (!s || !desc || !energy_out || !cut_out || !ticket || n < 1 || m < 0 ||
            (m > 0 && (!u || !v || !val)) || desc->steps < 1 || desc->trials < 1) {
            set_error("psa_server_submit: invalid arguments");
            return PSA_EINVAL;
        }
        std::unique_ptr<ServerJob> j(new ServerJob());
        j->n = n;
        j->u.assign(u, u + m);
        j->v.assign(v, v + m);
        j->val.assign(val, val + m);
        if (h) j->h.assign(h, h + n);
        j->graph_flags = graph_flags;
        j->desc = *desc;
        if (desc->i0) j->i0.assign(desc->i0, desc->i0 + desc->steps);
        if (desc->lambda) j->lambda.assign(desc->lambda, desc->lambda + n);
        if (desc->delta) j->delta.assign(desc->delta, desc->delta + n);
        if (desc->thr24) j->thr24.assign(desc->thr24, desc->thr24 + n);
        j->energy_out = energy_out;
        j->cut_out = cut_out;
        j->spins_out = spins_out;
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            set_error("psa_server_submit: server is shutting down");
            return PSA_ECANCELED;
        }
        if (s->opts.max_waiting > 0 && static_cast<int64_t>(s->waiting.size()) >= s->opts.max_waiting) {
            set_error("psa_server_submit: " + std::to_string(s->waiting.size()) +
                      " jobs already wait for admission (max_waiting); submit again later");
            return PSA_EAGAIN;
        }
        j->ticket = s->next_ticket++;
        j->submit_us = s->now_us();
        *ticket = j->ticket;
        s->waiting.push_back(j.get());
        s->to_prepare.push_back(j.get());
        s->jobs.emplace(j->ticket, std::move(j));
        s->cv_prep.notify_one();
        return PSA_OK;
    });
}

psa_status psa_server_poll(psa_server *s, uint64_t ticket, psa_result *out) {
    return psa::guarded("psa_server_poll", [&]() -> psa_status {
        if (!s || !out) {
            set_error("psa_server_poll: NULL argument");
            return PSA_EINVAL;
        }
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) {
            set_error("psa_server_poll: unknown ticket");
            return PSA_EINVAL;
        }
        fill_result(it->second.get(), out);
        if (it->second->status == PSA_JOB_ERROR) set_error(it->second->message);
        return PSA_OK;
    });
}

psa_status psa_server_wait(psa_server *s, uint64_t ticket, int64_t timeout_us, psa_result *out) {
    return psa::guarded("psa_server_wait", [&]() -> psa_status {
        if (!s || !out) {
            set_error("psa_server_wait: NULL argument");
            return PSA_EINVAL;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) {
            set_error("psa_server_wait: unknown ticket");
            return PSA_EINVAL;
        }
        ServerJob *j = it->second.get();
        auto done = [j] { return j->status >= PSA_JOB_DONE; };
        if (timeout_us < 0)
            s->cv_done.wait(lk, done);
        else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
            fill_result(j, out);
            set_error("psa_server_wait: timed out");
            return PSA_ETIMEDOUT;
        }
        fill_result(j, out);
        if (j->status == PSA_JOB_ERROR) set_error(j->message);
        return PSA_OK;
    });
}

psa_status psa_server_cancel(psa_server *s, uint64_t ticket) {
    return psa::guarded("psa_server_cancel", [&]() -> psa_status {
        if (!s) {
            set_error("psa_server_cancel: NULL argument");
            return PSA_EINVAL;
        }
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) {
            set_error("psa_server_cancel: unknown ticket");
            return PSA_EINVAL;
        }
        it->second->cancel = true;
        s->cv_work.notify_one();
        return PSA_OK;
    });
}

psa_status psa_server_release(psa_server *s, uint64_t ticket) {
    return psa::guarded("psa_server_release", [&]() -> psa_status {
        if (!s) {
            set_error("psa_server_release: NULL argument");
            return PSA_EINVAL;
        }
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end() || it->second->status < PSA_JOB_DONE) {
            set_error("psa_server_release: unknown or unfinished ticket");
            return PSA_EINVAL;
        }
        s->jobs.erase(it);
        return PSA_OK;
    });
}

psa_status psa_server_stats_get(psa_server *s, psa_server_stats *out) {
    return psa::guarded("psa_server_stats_get", [&]() -> psa_status {
        if (!s || !out) {
            set_error("psa_server_stats_get: NULL argument");
            return PSA_EINVAL;
        }
        std::lock_guard<std::mutex> g(s->mu);
        out->waiting = static_cast<int32_t>(s->waiting.size());
        out->resident = static_cast<int32_t>(s->resident.size());
        out->completed = s->completed;
        out->failed = s->failed;
        out->canceled = s->canceled;
        out->quanta = s->quanta;
        out->used_bytes = static_cast<int64_t>(s->used_bytes);
        out->budget_bytes = s->opts.hbm_budget_bytes;
        out->peak_resident = s->peak_resident;
        out->peak_used_bytes = static_cast<int64_t>(s->peak_used);
        return PSA_OK;
    });
}

void psa_server_destroy(psa_server *s) {
    if (!s) return;
    try {
        psa::server_shutdown(s);
    } catch (...) {
        psa::set_error_static("psa_server_destroy: exception while stopping the server");
    }
}

}  // extern "C"

namespace psa {

// Stop the server: cancel queued and resident jobs, join its threads, free it.
void server_shutdown(psa_server *s) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->to_prepare.clear();
        for (ServerJob *j : s->resident) j->cancel = true;  // retired after the current quantum
        s->cv_work.notify_all();
        s->cv_prep.notify_all();
    }
    for (std::thread &t : s->preparers)
        if (t.joinable()) t.join();
    if (s->worker.joinable()) s->worker.join();
    for (ServerJob *j : s->resident) release_device(j);
    delete s;
}

}  // namespace psa
