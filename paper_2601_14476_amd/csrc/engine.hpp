// engine.hpp -- internal objects of libpsa and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "psa.h"

namespace psa {

// Purpose tag of the variability draw in the Philox counter (the device
// kernels use tags 0 = initial spin, 1 = r, 2 = timing gate).
constexpr uint32_t kTagVarHost = 3u;
// thr24 value of a p-bit that fires on every step.
constexpr uint32_t kGateOneHost = 1u << 24;

// Thread-local error text behind psa_last_error().
void set_error(const std::string &msg);
void clear_error();
// Set the error text without allocating (a string literal, kept by address):
// the fallback when building the message itself fails.
void set_error_static(const char *msg) noexcept;

// Run the body of an exported call so that no exception unwinds across the C
// ABI: std::bad_alloc and std::length_error become PSA_ENOMEM, any other
// exception PSA_EINTERNAL, each with the error text set.
template <typename F>
psa_status guarded(const char *call, F &&body) noexcept {
    const char *what = nullptr;
    psa_status st = PSA_EINTERNAL;
    try {
        return body();
    } catch (const std::bad_alloc &) {
        st = PSA_ENOMEM;
        what = "host memory allocation failed";
    } catch (const std::length_error &) {
        st = PSA_ENOMEM;
        what = "host memory allocation failed (size too large)";
    } catch (const std::exception &e) {
        what = e.what();
    } catch (...) {
        what = "unknown exception";
    }
    try {
        set_error(std::string(call) + ": " + what);
    } catch (...) {
        set_error_static(st == PSA_ENOMEM ? "host memory allocation failed"
                                          : "internal error (exception in the host runtime)");
    }
    return st;
}

// Record a failed HIP call as the last error.
inline psa_status hip_fail(hipError_t err, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(err));
    return PSA_EHIP;
}

#define PSA_HIP(expr, what)                                    \
    do {                                                       \
        const hipError_t psa_hip_e_ = (expr);                  \
        if (psa_hip_e_ != hipSuccess) return psa::hip_fail(psa_hip_e_, what); \
    } while (0)

// Shape class of a tuning problem (tune.cpp).
using TuneKey = std::array<int64_t, 7>;

// Device copy of a graph in CSR form.  Row i holds its neighbours j in
// increasing order with their couplings J_ij.  Per-p-bit arrays are padded to
// n4 = 4 ceil(n/4) entries (h = 0) and row_ptr to n4 + 4 entries (padding rows
// are empty).  Packed copies of the edges, when the graph allows them:
//   pk32[e] = col | J << 16              (n <= 65536, |J| < 2^15)
//   pk16[e] = col << 1 | (J < 0)         (every |J| == 1, n <= 32768)
//   ux16[e] = col + (J < 0 ? n4 : 0)     (every |J| == 1, 2 n4 <= 65536)
struct DevGraph {
    int32_t n = 0;
    int32_t n4 = 0;
    int64_t nnz = 0;
    int32_t max_degree = 0;
    const int32_t *row_ptr = nullptr;  // [n4+4]
    const int32_t *col = nullptr;      // [nnz]
    const int32_t *val = nullptr;      // [nnz]
    const uint32_t *pk32 = nullptr;    // [nnz] or null
    const uint16_t *pk16 = nullptr;    // [nnz] or null
    const uint16_t *ux16 = nullptr;    // [nnz] or null
    // unit weights, degree <= 255: per-task ELL rows for the four-trial sweep
    // streaming edges from device memory; group g = eptr[m] .. eptr[m+1]-1 of
    // task m holds entry j of rows 4m..4m+3 as col | (J < 0) << 31, past a
    // row's end the zero word n4
    const uint32_t *ell = nullptr;     // [4 * groups] or null
    const int32_t *eptr = nullptr;     // [n4/4 + 1] or null
    const int32_t *h = nullptr;        // [n4]
    int64_t w2 = 0;                    // sum_i sum_j J_ij = 2 sum_{i<j} J_ij
};

// Device state of one run.  Spins are int8 in {-1,+1}, [n][t4] with the
// trial index innermost; t4 = trials rounded up to a multiple of 4, so the
// four trials 4q..4q+3 of p-bit i form one aligned 32-bit word.
struct DevRun {
    int32_t trials = 0;
    int32_t t4 = 0;
    int32_t steps = 0;
    uint32_t key0 = 0, key1 = 0;          // Philox key = 64-bit seed
    const float *i0 = nullptr;            // [steps]
    const float *lambda = nullptr;        // [n4]
    const float *delta = nullptr;         // [n4]
    const uint32_t *thr24 = nullptr;      // [n4] (padding p-bits: 0, never fire)
    int8_t *spins = nullptr;              // [n][t4]
    float *xs = nullptr;                  // SpSA held inputs [t4/4][n4][4], else nullptr
    uint32_t stall24 = 0;                 // SpSA stall threshold
    int32_t *ring = nullptr;              // TApSA windows [t4/4][n4][alpha][4], else nullptr
    int32_t alpha = 1;                    // TApSA window
    int32_t t_res = 0;                    // period mode: sub-steps per cycle (thr24 holds periods)
    // per-p-bit constants [n4][4] of the ELL four-trial sweep: h_i - deg_i,
    // lambda_i and delta_i (float bits), thr24_i
    const int32_t *pp = nullptr;
};

// How the persistent anneal kernel is launched for one run.
enum CsrKind : int32_t { kCsrPair = 0, kCsrPack32 = 1, kCsrPack16 = 2, kCsrUnit = 3 };
struct AnnealPlan {
    int32_t dense = 0;        // 1: dense int8 matrix-core path (nb below)
    int32_t nb = 4;           // dense path: 16-trial blocks per workgroup
    int32_t tpw = 1;          // trials per workgroup: 1 or 4
    int32_t lpt = 1;          // lanes per 4-p-bit task (tpw == 1): 1, 2 or 4
    int32_t csr = kCsrPair;   // edge encoding read by the kernel
    int32_t csr_lds = 0;      // 1: CSR, biases and per-p-bit factors staged in LDS
    int32_t block = 256;      // threads per workgroup
    int32_t grid = 0;         // workgroups
    size_t lds_bytes = 0;     // dynamic LDS per workgroup
};

// Arguments of one run as the anneal kernels read them.
struct AnnealArgs {
    int32_t n, n4, t4, t_begin, t_end, nnz, tasks;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *val;
    const uint32_t *pk32;
    const uint16_t *pk16;
    const uint16_t *ux16;
    const uint32_t *ell;
    const int32_t *eptr;
    const int32_t *pp;
    const int32_t *h;
    const float *i0;
    const float *lam;
    const float *dlt;
    const uint32_t *thr;
    const int32_t *order;
    uint32_t k0, k1;
    int8_t *spins;
    // SpSA (Eq. 5): held pre-activations [t4/4][n4][4] (nullptr = off) and the
    // stall threshold (an input is held iff (stall word >> 8) < stall24)
    float *xs;
    uint32_t stall24;
    // TApSA (Eq. 4): field windows [t4/4][n4][alpha][4] (nullptr = off)
    int32_t *ring;
    int32_t alpha;
    // period mode (t_res >= 1): thr holds integer periods, t_res sub-steps per step
    int32_t t_res;
};

// Kernel variants a batched launch can mix (one trial per workgroup).
enum BatchVariant : int32_t {
    kBatchUnitLds2 = 0,
    kBatchUnitGlb2 = 1,
    kBatchUnitLds4 = 2,
    kBatchUnitGlb4 = 3,
    kBatchP32Lds2 = 4,
    kBatchP32Glb2 = 5,
    kBatchPairGlb2 = 6,
    // four trials per workgroup (work item = group of four trials)
    kBatchP16Lds4T = 7,
    kBatchP16Glb4T = 8,
    kBatchP32Lds4T = 9,
    kBatchP32Glb4T = 10,
    kBatchPairGlb4T = 11,
};

// One run of a batched launch, as stored in the device job table.
struct BatchJob {
    AnnealArgs a;
    int32_t variant;
};

// Encodings of the dense coupling matrix (dense.hip): int8 entries (np a
// multiple of 128, int8 spins), 2-bit fields f in {0, +1, -1} with J =
// scale * f, or 1-bit fields f in {0, 1} with J = scale * f (every coupling
// the same value; np a multiple of 256 and fp4 spins for both).
enum : int32_t { kDenseI8 = 0, kDenseT2 = 1, kDenseB1 = 2 };
constexpr int32_t kDenseEncodings = 3;
constexpr bool dense_fp4(int32_t enc) { return enc != kDenseI8; }

// One run of the dense matrix-core path (dense.hip), as the step kernel reads
// it.  J is the encoded [np][np] coupling matrix; m0 / m1 are the two spin
// buffers (trial-major, [tp][np] int8 or [tp][np / 2] bytes of fp4); steps
// t .. t_end-1 of the launch sequence.
struct DenseJob {
    int32_t n, n4, np, t4, tp, t, t_end;
    int32_t scale;  // J = scale * entry (1 for int8)
    int32_t items;  // work items of the run in its work list (one step)
    const void *J;
    int8_t *m0, *m1;
    const int32_t *h;
    const float *i0;
    const float *lam;
    const float *dlt;
    const uint32_t *thr;
    uint32_t k0, k1;
    float *xs;         // SpSA held inputs [t4/4][n4][4], else nullptr
    uint32_t stall24;  // SpSA stall threshold
    int32_t *ring;     // TApSA windows [t4/4][n4][alpha][4], else nullptr
    int32_t alpha;     // TApSA window
    int32_t t_res;     // period mode: sub-steps per step (thr holds periods); 0 otherwise
};

// Period-mode sweep (period.hip): p-bits sorted by period into classes.
// Record of the p-bit at one sorted position (32 bytes, two 16-byte loads):
// its index, row bounds, bias and factors.
struct PeriodRec {
    int32_t i, rp0, rp1, h;
    float lam, dlt;
    int32_t cls, pad;  // class index (its period's rank)
};
// A class: the p-bits of one period, positions begin .. end-1.
struct PeriodClass {
    uint32_t period;
    int32_t begin, end, pad;
};
constexpr int32_t kPeriodMaxClasses = 64;  // one countdown per lane of a wavefront
struct PeriodPlan {
    int32_t nclass = 0;      // 0: the run does not take the period sweep
    int32_t block = 256;
    int32_t in_lds = 0;      // edges (and for the class sweep, records) in LDS
    int32_t pk32 = 0;        // edges read as col | J << 16 (else col, val)
    int32_t sbuf = 0;        // bytes per LDS spin buffer
    // resident lanes: lane l owns sorted positions l K .. l K + K - 1 with
    // their first `cache` edge words in registers (K = 0: class sweep)
    int32_t resident_k = 0;
    int32_t cache = 0;
    int32_t unit = 0;        // resident lanes: every |J| == 1 (negated spin copies)
    size_t lds_bytes = 0;
};
// Plan the period sweep of a one-trial-per-workgroup run (false: more than
// kPeriodMaxClasses distinct periods, no edges, or the spins do not fit in
// LDS; block_req 256, 512 or 1024 sets the block, else automatic) and
// build its records and classes from the host copies of the graph and factors.
bool plan_period(const DevGraph &g, const DevRun &run, const std::vector<int32_t> &row_ptr_host,
                 const std::vector<int32_t> &col_host, const std::vector<int32_t> &val_host,
                 const std::vector<int32_t> &h_host, const std::vector<float> &lam,
                 const std::vector<float> &dlt, const std::vector<uint32_t> &periods, size_t max_lds,
                 int32_t block_req, PeriodPlan *plan, std::vector<PeriodRec> *recs,
                 std::vector<PeriodClass> *classes, std::vector<uint32_t> *ecache);
// Steps t_begin .. t_end-1 (t_res sub-steps each), one workgroup per trial;
// ecache: the resident lanes' edge words ([n][cache], col | J << 16).
hipError_t launch_period(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const PeriodPlan &plan, const PeriodRec *recs, const PeriodClass *classes,
                         const uint32_t *ecache, int32_t t_begin, int32_t t_end);

// Choose tpw / lanes per task / CSR placement / block for a run
// (tpw_req, lpt_req, block_req: 0 = automatic).  Returns false with a reason if n does not fit in LDS.
bool plan_anneal(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                 int32_t block_req, size_t max_lds, int32_t num_cu, AnnealPlan *plan,
                 std::string *why);

// How a dense quantum is launched (psa_ctx_set_dense_launch, PSA_DENSE_LAUNCH_*).
enum : int32_t { kDenseLaunchSteps = PSA_DENSE_LAUNCH_STEPS, kDenseLaunchGraph = PSA_DENSE_LAUNCH_GRAPH,
                 kDenseLaunchPersistent = PSA_DENSE_LAUNCH_PERSISTENT };
constexpr uint32_t kDenseMaxPolls = 1u << 20;  // bound of one dependency wait (about a second)

// A captured dense step sequence: `steps` launches over one work list slice.
// The launches differ only in their step offset and take device pointers to
// the job table and work list, which the kernels read when they run; so the
// graph serves every later call of the same shape whatever the table holds.
struct DenseGraph {
    const DenseJob *table;
    const int4 *work;
    int32_t nwork, nb, enc, mode, steps;
    hipGraphExec_t exec;
};
constexpr size_t kDenseGraphCache = 8;    // graphs kept per context
constexpr int32_t kDenseGraphMinSteps = 2;

// Dense path launchers (dense.hip).  launch_dense_steps issues `steps`
// launches; launch s advances every run of the work list (job, 256-row group,
// trial tile of 16 nb; job -1 = empty slot) by its step t + s.  All runs of
// one work list share the encoding `enc`; `mode` 1 (plain) may be set only
// when every run of the list is pSA without held inputs, windows or periods,
// 2 (identity) only when besides every p-bit has lambda = 1, delta = 0 and
// thr24 >= 2^24 (no timing gate); 0 tests each run's mode at run time.
hipError_t launch_dense_steps(hipStream_t stream, const DenseJob *jobs, const int4 *work,
                              int32_t nwork, int32_t nb, int32_t enc, int32_t mode, int32_t steps);
// The same `steps` steps in one launch (dense_steps_kernel): the work list
// split into kDenseQueues queues of whole runs (queue x: items off[x] ..
// off[x+1]-1), tasks taken in step order from each queue's ticket counter,
// each waiting for its run's previous step (items of a run counted in
// DenseJob::items).  mode 1 or 2 only (plain pSA runs).  sync:
// dense_sync_words(table size) words, zeroed here first; its error flag
// (word 32 kDenseQueues) is left nonzero if a wait passed max_polls.
constexpr int32_t kDenseQueues = 8;  // one per XCD
struct DenseQueues {
    int32_t off[kDenseQueues + 1];
};
int32_t dense_sync_words(int32_t jobs);
hipError_t launch_dense_persistent(hipStream_t stream, const DenseJob *jobs, const int4 *work,
                                   const DenseQueues &q, int32_t nb, int32_t enc, int32_t mode, int32_t steps,
                                   uint32_t *sync, int32_t sync_words, uint32_t max_polls, int32_t num_cu);
// [n][t4] spins <-> one dense spin buffer of encoding enc
hipError_t launch_to_dense(hipStream_t stream, int32_t enc, int32_t n, int32_t t4, int32_t np, int32_t tp,
                           const int8_t *spins, int8_t *m);
hipError_t launch_from_dense(hipStream_t stream, int32_t enc, int32_t n, int32_t t4, int32_t np,
                             const int8_t *m, int8_t *spins);

// Kernel launchers (kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_init_spins(hipStream_t stream, int32_t n, const DevRun &run);
// Order in which a workgroup visits the tasks (groups of 4 p-bits): heaviest
// rows first, so that the lanes of a wavefront walk rows of similar length.
void task_order(const DevGraph &g, const std::vector<int32_t> &row_ptr_host,
                const AnnealPlan &plan, std::vector<int32_t> *order);
hipError_t launch_anneal(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const AnnealPlan &plan, const int32_t *order, int32_t t_begin,
                         int32_t t_end);
void fill_anneal_args(AnnealArgs *a, const DevGraph &g, const DevRun &run, const int32_t *order,
                      int32_t t_begin, int32_t t_end);
// Plan of one run inside a batched launch (tpw_req 4: four trials per
// workgroup; otherwise one, with lpt_req 4 or 2 lanes per task); sets the
// variant the batch kernel dispatches to.
bool plan_batch_item(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                     size_t max_lds, AnnealPlan *plan, int32_t *variant, std::string *why);
// One launch over a work list: work[b] = (index into jobs, trial), or
// (-1, 0) for an empty slot.
hipError_t launch_anneal_batch(hipStream_t stream, const BatchJob *jobs, const int2 *work,
                               int32_t nwork, int32_t block, size_t lds_bytes);
hipError_t launch_local_field(hipStream_t stream, const DevGraph &g,
                              const DevRun &run, int32_t *out_tn);
// Bytes of the per-block partial sums launch_energy_cut needs.
size_t energy_partial_bytes(int32_t n, int32_t t4);
hipError_t launch_energy_cut(hipStream_t stream, const DevGraph &g, const DevRun &run,
                             int64_t *part, int64_t *energy, int64_t *cut);
// One run of a batched energy / cut read-out: its graph and spins, its share
// of the partial-sum buffer (energy_partial_bytes of it) and its outputs.
// wg0: its first workgroup of the partial pass (energy_batch_wgs of them);
// k0: its first thread of the final pass (one per trial); lpr: lanes that
// share a row in the partial pass (1, 4 or 16, by the mean degree).
struct EnergyJob {
    int32_t n = 0, t4 = 0, trials = 0, blocks = 0;
    int32_t wg0 = 0, k0 = 0, lpr = 1;
    int64_t w2 = 0;
    const int32_t *row_ptr = nullptr, *col = nullptr, *val = nullptr, *h = nullptr;
    const int8_t *spins = nullptr;
    int64_t *part = nullptr;
    int64_t *energy = nullptr, *cut = nullptr;
};
// The read-outs of `count` runs (a device table, wg0 and k0 ascending) in two
// launches: wgs = the runs' partial workgroups, trials = their trials.
hipError_t launch_energy_cut_batch(hipStream_t stream, const EnergyJob *jobs, int32_t count, int32_t wgs,
                                   int32_t trials);
// Workgroups of one run's batched partial pass: row blocks x chunks of 16 trials.
inline int64_t energy_batch_wgs(int32_t n, int32_t t4) {
    return static_cast<int64_t>((n + 255) / 256) * ((t4 / 4 + 3) / 4);
}
hipError_t launch_spins_to_tn(hipStream_t stream, int32_t n, const DevRun &run,
                              int8_t *out_tn);
hipError_t launch_spins_from_tn(hipStream_t stream, int32_t n, const DevRun &run,
                                const int8_t *in_tn);
// Test entry points: device tanh_f32 of count values; pbit_up decisions of
// count (x, word) pairs with the branch taken (bit 0 up, bit 1 tanh_f32).
hipError_t launch_debug_tanh(hipStream_t stream, int64_t count, const float *x, float *y);
hipError_t launch_debug_decide(hipStream_t stream, int64_t count, const float *x,
                               const uint32_t *word, uint8_t *out);

// Host-side helpers (host_params.cpp).
void philox4x32_10_host(const uint32_t ctr[4], uint32_t key0, uint32_t key1,
                        uint32_t out[4]);
psa_status fill_schedule(int32_t steps, double i0_min, double i0_max, float *out);
psa_status draw_variability(int32_t n, uint64_t seed, double sigma_lambda,
                            double sigma_delta, double sigma_nu, double p_mean,
                            float *lambda, float *delta, uint32_t *thr24);
// Integer timing periods of the period mode (psa_periods_draw).
psa_status draw_periods(int32_t n, uint64_t seed, double sigma_nu, int32_t t_res,
                        uint32_t *period);

// Graph ingestion (graph.cpp): CPU phase, then device upload.
struct HostGraph {
    psa_graph_info info{};
    int32_t n = 0, n4 = 0, max_degree = 0;
    int64_t nnz = 0, w2 = 0;
    std::vector<int32_t> rp32;  // [n4+4]
    std::vector<int32_t> col, val;
    std::vector<int32_t> h;     // [n4]
    std::vector<uint32_t> pk32;
    std::vector<uint16_t> pk16, ux16;
    std::vector<uint32_t> ell;
    std::vector<int32_t> eptr;
};
psa_status host_graph_from_edges(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                                 const int32_t *val, const int32_t *h, uint32_t flags,
                                 HostGraph *out);
psa_status host_graph_from_csr(int32_t n, const int64_t *row_ptr, const int32_t *col,
                               const int32_t *val, const int32_t *h, uint32_t flags,
                               HostGraph *out);
psa_status upload_graph(psa_ctx *ctx, HostGraph &&hg, psa_graph **out);
void graph_release(psa_graph *g);   // free now (creation failures)
void graph_unref(psa_graph *g);     // drop one reference, free at zero
// Chip figures of the cost model (MI355X: 256 CUs at 2.4 GHz).
constexpr double kValuOpsPerSecond = 256.0 * 4 * 16 * 2.4e9;  // 32-bit lane-ops
constexpr double kMfmaI8OpsPerSecond = 5.0e15;                // dense int8
constexpr double kMfmaF4OpsPerSecond = 10.1e15;               // dense fp4
constexpr double kHbmBytesPerSecond = 8.0e12;
// Modelled seconds per step of the CSR sweep (with the given plan) and of the
// dense matrix-core step (1-bit, 2-bit or int8 couplings).
double csr_step_seconds(const DevGraph &g, const DevRun &run, const AnnealPlan &plan);
double dense_step_seconds(int32_t n, int32_t t4, bool two_bit, bool one_bit);
// True when every stored coupling has one magnitude (the 2-bit encoding).
bool dense_two_bit(const psa_graph *g);
// Every stored coupling the same nonzero value (the 1-bit dense encoding).
bool dense_one_bit(const psa_graph *g);
// Cost model of the automatic path choice: dense when the rows are long
// enough that the matrix-core product beats the CSR walk, and the couplings
// have a dense encoding.
bool prefer_dense(const psa_graph *g, const DevRun &run, const AnnealPlan &plan);
// Build and upload the dense int8 coupling matrix of g (once); EUNSUPPORTED
// if a coupling does not fit int8.
psa_status ensure_dense_matrix(psa_graph *g);
// Free the dense coupling matrix of g (after the work queued on the context's
// streams), for a graph that no live job reads it through.
void release_dense_matrix(psa_graph *g);
// Advance the dense-planned jobs of `jobs` by up to k steps (each clipped to
// its schedule) on the context's second stream; the caller joins it.
// share: the fraction of the device's compute units a persistent dense launch
// may fill (the rest is left to a CSR batch launched beside it).
psa_status dense_step_jobs(psa_ctx *ctx, psa_job *const *jobs, int32_t count, int32_t k, double share = 1.0);

// Path and launch shape of d from the context's tuning cache, measured on a
// miss (mode PSA_TUNE_ALONE or PSA_TUNE_BATCH); clears PSA_TUNE (tune.cpp).
psa_status tuned_desc(psa_ctx *ctx, const psa_graph *g, psa_run_desc *d, uint32_t mode);

// Per-family timing (abi.cpp): begin/end a span on `stream` when the
// context records timing (no-ops otherwise).
enum : int { kTimeAnneal = 0, kTimeBatch = 1, kTimeDense = 2 };
psa_status time_begin(psa_ctx *ctx, hipStream_t stream, hipEvent_t *ev);
psa_status time_end(psa_ctx *ctx, hipStream_t stream, int family, hipEvent_t begin,
                    int64_t launches);

// Static device scratch of psa_anneal_noalloc (noalloc.hip): look up the
// array's address on `device` (which must be current) once and keep it;
// noalloc_scratch returns it (nullptr before the lookup).
psa_status noalloc_scratch_init(int32_t device);
void *noalloc_scratch(int32_t device);

// A scratch copy of `src` for timing (abi.cpp): the same run and plan, its
// own spins (initial state), input-stage state and dense spin buffers; the
// read-only run arrays are shared with src, which must outlive it.
psa_status clone_job_for_timing(psa_job *src, psa_job **out);

// Context references (abi.cpp).
void ctx_retain(psa_ctx *ctx);
void ctx_release(psa_ctx *ctx);

// XCD-aware work list of a batched launch (batch.cpp).
void build_work_list(const std::vector<int32_t> &trials, const std::vector<double> &cost,
                     std::vector<int2> *work);

}  // namespace psa

struct psa_ctx {
    // references: the creator's plus one per live graph and job; the context
    // is freed when the last one is dropped (psa_ctx_destroy drops the
    // creator's), so objects may be destroyed in any order
    std::atomic<int32_t> refs{1};
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t num_cu = 0;
    size_t max_lds = 0;
    // staging of batched launches (grow-only; reused after a stream sync)
    void *d_batch_table = nullptr, *d_batch_work = nullptr;
    size_t batch_table_cap = 0, batch_work_cap = 0;
    std::vector<psa::BatchJob> h_batch_table;
    std::vector<int2> h_batch_work;
    // batched energy / cut read-outs: the run table (grow-only)
    void *d_energy_table = nullptr;
    size_t energy_table_cap = 0;
    std::vector<psa::EnergyJob> h_energy_table;
    // dense-path launches run on a second stream, joined with events
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // a second coupling encoding's step-by-step sequence runs on a third
    // stream beside the first encoding's, forked from and joined to stream2
    hipStream_t stream3 = nullptr;
    hipEvent_t ev_fork3 = nullptr, ev_join3 = nullptr;
    void *d_dense_table = nullptr, *d_dense_work = nullptr;
    size_t dense_table_cap = 0, dense_work_cap = 0;
    std::vector<psa::DenseJob> h_dense_table;
    std::vector<int4> h_dense_work;
    // how dense quanta are launched (psa_ctx_set_dense_launch); captured
    // step sequences (batch.cpp), most recently used last; the persistent
    // launch's counters (one region per encoding) and the pinned copy
    // of their error flags, checked at the next dense quantum
    int32_t dense_launch = psa::kDenseLaunchSteps;
    uint32_t dense_max_polls = psa::kDenseMaxPolls;
    std::vector<psa::DenseGraph> dense_graph_cache;
    uint32_t *d_dense_sync = nullptr;
    size_t dense_sync_cap = 0;
    uint32_t *h_dense_err = nullptr;  // [kDenseEncodings], pinned
    // per-family device timing (psa_ctx_set_timing): event pairs awaiting
    // resolution, by family 0 anneal, 1 batch, 2 dense
    bool timing = false;
    struct TimedSpan {
        int family;
        hipEvent_t begin, end;
        int64_t launches;
    };
    std::vector<TimedSpan> spans;
    std::vector<hipEvent_t> event_pool;
    double timed_ms[3] = {0.0, 0.0, 0.0};
    int64_t timed_launches[3] = {0, 0, 0};
    int64_t timed_graph_launches = 0;  // dense launches replayed from a captured graph
    // measured path / launch shape per shape class (psa_autotune)
    std::mutex tune_mu;
    std::map<psa::TuneKey, psa_tune_result> tune_cache;
};

struct psa_graph {
    psa_ctx *ctx = nullptr;
    bool retained = false;  // holds a reference on ctx
    // references: the creator's plus one per live job on this graph
    std::atomic<int32_t> refs{1};
    psa_graph_info info{};
    psa::DevGraph dev;
    // owning device pointers
    int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_val = nullptr, *d_h = nullptr;
    uint32_t *d_pk32 = nullptr;
    uint16_t *d_pk16 = nullptr, *d_ux16 = nullptr;
    uint32_t *d_ell = nullptr;
    int32_t *d_eptr = nullptr;
    std::vector<int32_t> row_ptr_host;  // [n4+4]
    std::vector<int32_t> h_host;        // [n4]
    std::vector<int32_t> col_host, val_host;  // for the dense matrix, on demand
    void *d_dense = nullptr;            // encoded [np][np] couplings, built on first use
    int32_t np = 0;                     // n rounded up to 128
    int32_t dense_enc = 0;              // kDenseI8, kDenseT2 or kDenseB1
    int32_t dense_scale = 1;            // J = dense_scale * entry
    size_t dev_bytes = 0;               // device bytes of the CSR and its encodings
    size_t dense_bytes = 0;             // device bytes of d_dense
};

struct psa_job {
    psa_ctx *ctx = nullptr;
    bool retained = false;         // holds a reference on ctx
    psa_graph *graph_ref = nullptr;  // holds a reference on its graph
    const psa_graph *g = nullptr;
    psa::DevRun run;
    int32_t t = 0;       // steps applied so far
    psa::AnnealPlan plan;
    int32_t *d_order = nullptr;  // [n4/4] task visiting order
    int8_t *d_m = nullptr;       // dense path: two [tp][np] buffers
    int32_t tp = 0;
    // owning device pointers
    float *d_i0 = nullptr, *d_lambda = nullptr, *d_delta = nullptr;
    uint32_t *d_thr24 = nullptr;
    int8_t *d_spins = nullptr;
    float *d_xs = nullptr;       // SpSA held inputs
    int32_t *d_ring = nullptr;   // TApSA field windows
    int32_t *d_pp = nullptr;     // per-p-bit constants of the ELL sweep
    // period-mode sweep (pplan.nclass > 0): records and classes
    psa::PeriodPlan pplan;
    psa::PeriodRec *d_prec = nullptr;
    psa::PeriodClass *d_pcls = nullptr;
    uint32_t *d_pcache = nullptr;  // resident lanes' edge words
    void *d_scratch = nullptr;   // read-out staging
    size_t scratch_bytes = 0;
    size_t dev_bytes = 0;        // device bytes of every allocation above
    // the device arrays above are carved from memory the job does not own
    // (psa_anneal_noalloc's static scratch): never freed or grown
    bool borrowed = false;
    // every p-bit has lambda = 1, delta = 0 and thr24 >= 2^24 (no timing gate)
    bool identity_factors = false;
    // a timing clone: schedule, factors, task order and period records are
    // another job's (kept alive by `shares`); only the spin and input-stage
    // state and the staging are its own
    psa_job *shares = nullptr;
};
