// engine.hpp -- internal objects of libpsa and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Device copy of a graph in CSR form.  Row i holds its neighbours j in
// increasing order with their couplings J_ij; h is never null (zeros).
// Packed copies of the same entries, when the graph allows them:
//   pk32[e] = col | J << 16           (n <= 65536, |J| < 2^15)
//   pk16[e] = col << 1 | (J < 0)      (every |J| == 1, n <= 32768)
struct DevGraph {
    int32_t n = 0;
    int64_t nnz = 0;
    const int32_t *row_ptr = nullptr;  // [n+1]
    const int32_t *col = nullptr;      // [nnz]
    const int32_t *val = nullptr;      // [nnz]
    const uint32_t *pk32 = nullptr;    // [nnz] or null
    const uint16_t *pk16 = nullptr;    // [nnz] or null
    const int32_t *h = nullptr;        // [n]
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
    const float *lambda = nullptr;        // [n]
    const float *delta = nullptr;         // [n]
    const uint32_t *thr24 = nullptr;      // [n]
    int8_t *spins = nullptr;              // [n][t4]
};

// How the persistent anneal kernel is launched for one run.
enum CsrKind : int32_t { kCsrPair = 0, kCsrPack32 = 1, kCsrPack16 = 2 };
struct AnnealPlan {
    int32_t tpw = 1;          // trials per workgroup: 1 or 4
    int32_t lpt = 1;          // lanes per 4-p-bit task (tpw == 1): 1, 2 or 4
    int32_t csr = kCsrPair;   // edge encoding read by the kernel
    int32_t csr_lds = 0;      // 1: CSR, biases and per-p-bit factors staged in LDS
    int32_t block = 256;      // threads per workgroup
    int32_t grid = 0;         // workgroups
    size_t lds_bytes = 0;     // dynamic LDS per workgroup
};

// Choose tpw / lanes per task / CSR placement / block for a run
// (tpw_req, lpt_req, block_req: 0 = automatic).  Returns false with a reason if n does not fit in LDS.
bool plan_anneal(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                 int32_t block_req, size_t max_lds, int32_t num_cu, AnnealPlan *plan,
                 std::string *why);

// Kernel launchers (kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_init_spins(hipStream_t stream, int32_t n, const DevRun &run);
hipError_t launch_anneal(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const AnnealPlan &plan, int32_t t_begin, int32_t t_end);
hipError_t launch_local_field(hipStream_t stream, const DevGraph &g,
                              const DevRun &run, int32_t *out_tn);
hipError_t launch_energy_cut(hipStream_t stream, const DevGraph &g,
                             const DevRun &run, int64_t *energy, int64_t *cut);
hipError_t launch_spins_to_tn(hipStream_t stream, int32_t n, const DevRun &run,
                              int8_t *out_tn);
hipError_t launch_spins_from_tn(hipStream_t stream, int32_t n, const DevRun &run,
                                const int8_t *in_tn);

// Host-side helpers (host_params.cpp).
void philox4x32_10_host(const uint32_t ctr[4], uint32_t key0, uint32_t key1,
                        uint32_t out[4]);
psa_status fill_schedule(int32_t steps, double i0_min, double i0_max, float *out);
psa_status draw_variability(int32_t n, uint64_t seed, double sigma_lambda,
                            double sigma_delta, double sigma_nu, double p_mean,
                            float *lambda, float *delta, uint32_t *thr24);

}  // namespace psa

struct psa_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t num_cu = 0;
    size_t max_lds = 0;
};

struct psa_graph {
    psa_ctx *ctx = nullptr;
    psa_graph_info info{};
    psa::DevGraph dev;
    // owning device pointers
    int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_val = nullptr, *d_h = nullptr;
    uint32_t *d_pk32 = nullptr;
    uint16_t *d_pk16 = nullptr;
};

struct psa_job {
    psa_ctx *ctx = nullptr;
    const psa_graph *g = nullptr;
    psa::DevRun run;
    int32_t t = 0;       // steps applied so far
    psa::AnnealPlan plan;
    // owning device pointers
    float *d_i0 = nullptr, *d_lambda = nullptr, *d_delta = nullptr;
    uint32_t *d_thr24 = nullptr;
    int8_t *d_spins = nullptr;
    void *d_scratch = nullptr;   // read-out staging
    size_t scratch_bytes = 0;
};
