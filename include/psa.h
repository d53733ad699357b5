/*
 * psa.h -- C ABI of libpsa, an MI355X (gfx950) engine for p-bit simulated
 * annealing (pSA) with device variability on Ising models of MAX-CUT.
 *
 * Method: Onizawa & Hanyu, "GPU-accelerated simulated annealing based on
 * p-bits with real-world device-variability modeling", arXiv 2601.14476.
 *   - p-bit output            : Eq. 1, sigma_i(t+1) = sgn(r_i(t) + tanh(I_i(t)))
 *   - Ising energy            : Eq. 2, H = -sum h_i s_i - sum_{i<j} J_ij s_i s_j
 *   - p-bit input             : Eq. 3, I_i = I0 (h_i + sum_j J_ij s_j)
 *   - variability p-bit       : Eq. 6, intensity lambda_i, offset delta_i, timing nu_i
 *   - variability draws       : Eq. 7, lambda ~ N(1, sl^2), delta ~ N(0, sd^2), nu ~ N(0, sn^2)
 *   - schedule                : Methods (experimental conditions),
 *                               I0(t+1) = I0(t)/beta, beta = (I0min/I0max)^(1/(cycle-1)),
 *                               I0min = 0.1/mean(s_i), I0max = 10/mean(s_i)
 *   - SimulatedAnnealingModule: the pseudo-code listing of the update kernel
 *
 * What one step computes, for every trial k and p-bit i at once (all p-bits
 * read the spins of the previous step):
 *     L_i   = h_i + sum_j J_ij m_j                         (int32, exact)
 *     fire  = thr24_i >= 2^24  or  (u_gate >> 8) < thr24_i  (timing factor)
 *     x     = (I0[t] * lambda_i) * ((float)L_i + delta_i)   (FP32, this order)
 *     m_i'  = fire ? (tanh(x) > r ? +1 : -1) : m_i
 * with r uniform on the odd multiples of 2^-24 in (-1,1) and all random
 * words from Philox4x32-10 (key = seed, counter = (t, i/4, k, purpose),
 * word i mod 4).  Results are bit-identical for any launch geometry.
 *
 * Conventions
 *   - Every call returns a psa_status; on failure the outputs are left
 *     untouched and psa_last_error() describes the failure (thread-local).
 *   - Nothing throws across the ABI: every call catches what its C++ body
 *     throws (a failed host allocation becomes PSA_ENOMEM, any other
 *     exception PSA_EINTERNAL).  No call keeps a pointer it was given:
 *     host arrays are copied before the call returns.
 *   - "device pointer" arguments are HIP device addresses on the context's
 *     device (for instance torch.Tensor.data_ptr() of a cuda tensor); work
 *     on them is ordered on the context's stream.  Flags select whether an
 *     output pointer is host or device memory.
 *   - Objects (context, graph, job) are not thread-safe; use one per thread
 *     or serialise calls.
 */
#ifndef PSA_H
#define PSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t psa_status;
#define PSA_OK 0
#define PSA_EINVAL (-1)       /* bad argument or invalid graph          */
#define PSA_ENOMEM (-2)       /* host or device allocation failed        */
#define PSA_EHIP (-3)         /* a HIP runtime call failed               */
#define PSA_EUNSUPPORTED (-4) /* valid request the library cannot serve  */
#define PSA_EAGAIN (-5)       /* server queue full: submit again later   */
#define PSA_ECANCELED (-6)    /* the job was canceled                    */
#define PSA_ETIMEDOUT (-7)    /* a wait ended before the job finished    */
#define PSA_EINTERNAL (-8)    /* an unexpected failure inside the library
                                 (an exception of the host runtime, e.g.
                                 a thread that could not be started)     */

typedef struct psa_ctx psa_ctx;
typedef struct psa_graph psa_graph;
typedef struct psa_job psa_job;

/* ------------------------------------------------------------------ */
/* Context and errors                                                   */
/* ------------------------------------------------------------------ */

/* Library version string, e.g. "0.1.0 gfx950".  Static storage. */
const char *psa_version(void);

/* Thread-local text of the last failure on this thread ("" if none).
 * Valid until the next failing call on the same thread. */
const char *psa_last_error(void);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * owned by the caller (NULL = the context creates and owns one).  All
 * device work of objects made from this context is ordered on it. */
psa_status psa_ctx_create(int32_t device, void *hip_stream, psa_ctx **out);

/* Wait for all work queued on the context's stream. */
psa_status psa_ctx_synchronize(psa_ctx *ctx);

/* Drop the creator's reference to the context.  Graphs and jobs made from
 * it hold references of their own, so they may be destroyed before or after
 * the context; its streams and staging are released with the last
 * reference.  NULL is ignored. */
void psa_ctx_destroy(psa_ctx *ctx);

/* Device time per kernel family, measured with HIP events on the stream
 * each family is launched on (the context's stream for the CSR sweep and
 * batch kernels, its second stream for the dense step kernels).  Off by
 * default; psa_ctx_set_timing(ctx, 1) starts recording, and
 * psa_ctx_timing_read waits for the recorded work, fills *out with the
 * totals since the last read and clears them. */
typedef struct psa_timing {
    double anneal_ms;        /* CSR sweep launches (one job stepped alone) */
    double batch_ms;         /* CSR batch kernel launches                  */
    double dense_ms;         /* dense step sequences (launch gaps included) */
    int64_t anneal_launches;
    int64_t batch_launches;
    int64_t dense_launches;  /* per dense work list: one per step, or one
                                for a persistent quantum                    */
    int64_t dense_graph_launches; /* of dense_launches, those replayed from a
                                     captured graph (psa_ctx_set_dense_launch) */
} psa_timing;

psa_status psa_ctx_set_timing(psa_ctx *ctx, int32_t on);
psa_status psa_ctx_timing_read(psa_ctx *ctx, psa_timing *out);

/* How the dense path launches a quantum of k steps (k launches of the step
 * kernel that differ only in their step offset):
 *   PSA_DENSE_LAUNCH_STEPS (default)  one launch per step.
 *   PSA_DENSE_LAUNCH_PERSISTENT  one launch for all k steps.  Whole runs are
 *     dealt to 8 queues (one per XCD); workgroups take each queue's tasks in
 *     step order from its ticket counter, and a task waits until every item
 *     of its run has finished the previous step (a device counter per run;
 *     spins stored and read at device coherence, since a run's workgroups may
 *     sit on different XCDs with separate L2s).  A task only waits on tasks
 *     of its queue taken before it, by running workgroups, so the waits end
 *     however many workgroups the device keeps resident.  Beside a CSR batch
 *     (psa_jobs_step_batch) the launch takes the dense family's modelled
 *     share of the compute units.  Each wait is bounded (about a second); a
 *     wait past the bound makes the workgroups leave and the next dense
 *     quantum on the context return PSA_EHIP.  Measured on par with STEPS
 *     for dense runs alone, and slower beside a CSR batch (whose 1,024-thread
 *     workgroups need whole compute units that the resident dense
 *     workgroups keep partly occupied).
 *   PSA_DENSE_LAUNCH_GRAPH  the k launches captured once per shape (job table
 *     and work list addresses, work items, trial tile, encoding, epilogue
 *     mode, k) as a HIP graph and replayed for every later quantum of that
 *     shape, whatever jobs the table holds then (the kernels read it when
 *     they run); up to 8 graphs kept per context, least recently used
 *     evicted.  Measured slower than STEPS on this runtime.
 * Results are identical in every mode.  Leaving GRAPH frees the kept graphs
 * (after the dense stream drains).  EINVAL: ctx NULL or an unknown mode;
 * EHIP: a HIP call failed. */
#define PSA_DENSE_LAUNCH_STEPS 0
#define PSA_DENSE_LAUNCH_GRAPH 1
#define PSA_DENSE_LAUNCH_PERSISTENT 2
psa_status psa_ctx_set_dense_launch(psa_ctx *ctx, int32_t how);

/* ------------------------------------------------------------------ */
/* Graphs (Eq. 2-3: couplings J and biases h)                           */
/* ------------------------------------------------------------------ */

#define PSA_GRAPH_ISING 0u  /* edge values are couplings J_uv            */
#define PSA_GRAPH_MAXCUT 1u /* edge values are MAX-CUT weights w, J = -w */

typedef struct psa_graph_info {
    int32_t n;             /* p-bits                                      */
    int64_t edges;         /* undirected edges (pairs i<j with J_ij != 0) */
    int64_t nnz;           /* 2 * edges: stored directed entries          */
    int64_t w_total;       /* sum over edges of w_ij = -J_ij              */
    int32_t max_abs_field; /* max_i |h_i| + sum_j |J_ij|  (< 2^24)        */
    int32_t max_degree;    /* largest row length                          */
    int32_t unit_weights;  /* 1 if every |J_ij| == 1                      */
    double mean_s;         /* mean_i sqrt((n-1) Var(J_i,:)), dense rows   */
    int64_t device_bytes;  /* device memory the graph holds now: CSR,
                              packed encodings and, once a dense-path job
                              has built it, the dense coupling matrix
                              (0 from psa_graph_check_edges)              */
} psa_graph_info;

/* Build a graph from an undirected edge list on the host: edge e joins
 * u[e] and v[e] (0 <= u,v < n, u != v, each pair at most once) with value
 * val[e] (a coupling, or a MAX-CUT weight with PSA_GRAPH_MAXCUT).  h may be
 * NULL (all zero).  The arrays are copied; the graph is uploaded to the
 * context's device in CSR form.  EINVAL on self loops, repeated pairs,
 * indices out of range, or max_i |h_i| + sum_j |J_ij| >= 2^24 (which keeps
 * the float conversion of every field exact). */
psa_status psa_graph_from_edges(psa_ctx *ctx, int32_t n, int64_t m,
                                const int32_t *u, const int32_t *v,
                                const int32_t *val, const int32_t *h,
                                uint32_t flags, psa_graph **out);

/* Build a graph from a symmetric host CSR (row_ptr[n+1], col[nnz], val[nnz],
 * no diagonal, no repeated column in a row, val[i->j] == val[j->i]). */
psa_status psa_graph_from_csr(psa_ctx *ctx, int32_t n, const int64_t *row_ptr,
                              const int32_t *col, const int32_t *val,
                              const int32_t *h, uint32_t flags,
                              psa_graph **out);

psa_status psa_graph_info_get(const psa_graph *g, psa_graph_info *out);

/* The host half of psa_graph_from_edges without a context or device:
 * validate the edge list exactly as psa_graph_from_edges does (same EINVAL
 * cases) and return the graph's statistics (n, edges, W_total, mean(s_i),
 * bounds; device_bytes = 0).  PSA_ENOMEM if the host cannot hold the CSR
 * being built (about 24 bytes per edge).  Usable on a machine without a
 * GPU, e.g. to check requests before submitting them to a server. */
psa_status psa_graph_check_edges(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                                 const int32_t *val, const int32_t *h, uint32_t flags,
                                 psa_graph_info *out);

/* Drop the creator's reference; jobs on the graph keep it alive until they
 * are destroyed.  NULL is ignored. */
void psa_graph_destroy(psa_graph *g);

/* ------------------------------------------------------------------ */
/* Schedule (Methods, experimental conditions)                         */
/* ------------------------------------------------------------------ */

/* The paper's I0 endpoints for graph g: I0min = 0.1/mean(s_i),
 * I0max = 10/mean(s_i).  EINVAL if mean(s_i) == 0 (no couplings). */
psa_status psa_schedule_paper(const psa_graph *g, double *i0_min,
                              double *i0_max);

/* Fill host i0_out[steps] with I0(0) = i0_min, I0(t+1) = I0(t)/beta,
 * beta = (i0_min/i0_max)^(1/(steps-1)), evaluated in double and rounded to
 * float per step.  EINVAL unless steps >= 1 and 0 < i0_min <= i0_max. */
psa_status psa_schedule_fill(int32_t steps, double i0_min, double i0_max,
                             float *i0_out);

/* ------------------------------------------------------------------ */
/* Device variability (Eq. 6-7)                                         */
/* ------------------------------------------------------------------ */

/* Draw the per-p-bit factors once per run, on the host, from the run seed:
 *   lambda_i = 1 + sigma_lambda z1     (intensity, Eq. 7a)
 *   delta_i  = sigma_delta z2          (offset, Eq. 7b)
 *   p_i      = clip(p_mean + sigma_nu z3, 0, 1), thr24_i = floor(p_i 2^24)
 *              (timing, Eq. 7c, as a per-step update probability)
 * with z1..z3 standard normals (Box-Muller, cosine branch) from the Philox
 * words of counters (0, i, 0, 3) and (0, i, 1, 3).  Outputs are host
 * arrays of n entries.  EINVAL on negative sigmas or p_mean outside [0,1]. */
psa_status psa_variability_draw(int32_t n, uint64_t seed, double sigma_lambda,
                                double sigma_delta, double sigma_nu,
                                double p_mean, float *lambda_out,
                                float *delta_out, uint32_t *thr24_out);

/* Integer timing periods of the period mode: period_i = max(1,
 * rint(t_res (1 + sigma_nu z3))) with the same standard normal z3 as the
 * update probability of psa_variability_draw.  EINVAL on t_res < 1 or a
 * negative sigma. */
psa_status psa_periods_draw(int32_t n, uint64_t seed, double sigma_nu, int32_t t_res,
                            uint32_t *period_out);

/* ------------------------------------------------------------------ */
/* Runs                                                                  */
/* ------------------------------------------------------------------ */

/* Description of one anneal.  Optional host arrays (NULL = derived):
 *   i0[steps]              -- schedule; else psa_schedule_fill(i0_min, i0_max)
 *                             and, if i0_min <= 0, the paper's endpoints
 *   lambda/delta/thr24[n]  -- variability; else psa_variability_draw(...)
 * trials >= 1, steps >= 1.  Launch shape (results never depend on it):
 * `block` = threads per workgroup (0 = auto, else 256, 512 or 1024),
 * `trials_per_group` = trials one workgroup advances (0 = auto, 1 or 4) and
 * `lanes_per_task` = lanes sharing one group of four p-bits when a
 * workgroup advances one trial (0 = auto, 1, 2 or 4). */
typedef struct psa_run_desc {
    int32_t steps;
    int32_t trials;
    uint64_t seed;
    double i0_min;
    double i0_max;
    const float *i0;
    double sigma_lambda;
    double sigma_delta;
    double sigma_nu;
    double p_mean;
    const float *lambda;
    const float *delta;
    const uint32_t *thr24;
    int32_t block;
    int32_t trials_per_group;
    int32_t lanes_per_task;
    uint32_t flags; /* PSA_PATH_*, PSA_TUNE */
    uint32_t algorithm; /* PSA_ALG_PSA, PSA_ALG_SPSA or PSA_ALG_TAPSA */
    double p_stall;     /* SpSA: probability that an input is held (0..1) */
    int32_t window;     /* TApSA: steps averaged, alpha (1..64) */
    int32_t t_res;      /* 0: timing as an update probability; >= 1: timing
                           as integer periods of t_res sub-steps per cycle */
    const uint32_t *period; /* period mode, optional [n] periods (>= 1) */
} psa_run_desc;

/* Timing modes of the variability model (Eq. 6, nu_i):
 *   t_res = 0 (default): probability mode -- each step a p-bit fires with its
 *            probability thr24_i / 2^24 (gate word), else holds its output.
 *   t_res >= 1: period mode, the listing's count mod nu[i] gate -- a cycle
 *            (one step of the schedule) has t_res sub-steps tau = t t_res + s;
 *            at sub-step tau every p-bit whose period divides tau updates
 *            (synchronously, I0 of cycle t, r from Philox counter
 *            (tau, i/4, k, 1)); periods are max(1, rint(t_res (1 + nu_i))),
 *            nu_i ~ N(0, sigma_nu^2) (psa_periods_draw), unless given.
 *            Plain pSA only; steps * t_res must stay below 2^22. */

/* Update rule (psa_run_desc.algorithm).
 *   PSA_ALG_PSA   plain pSA (Eq. 3): every step forms the input of each
 *                 p-bit from the spins of the previous step.
 *   PSA_ALG_SPSA  stalled p-bits (Eq. 5): at each step t > 0 the input of a
 *                 p-bit (its whole pre-activation x = (I0 lambda)(L + delta)
 *                 of the step it was last formed) is held with probability
 *                 p_stall, else formed anew; step 0 always forms it.  The
 *                 stall of p-bit i, trial k at step t is decided by Philox
 *                 word i mod 4 of counter (t, i/4, k, 4): held iff
 *                 (word >> 8) < floor(p_stall 2^24).  The output rule
 *                 (timing gate, r, tanh) is unchanged.  A job keeps the held
 *                 inputs on the device (4 bytes per p-bit and trial).
 *   PSA_ALG_TAPSA time-averaged p-bits (Eq. 4): the input of a p-bit is I0
 *                 times the mean of its last `window` integer fields
 *                 TI(t) = h + sum_j J m_j(t) (of the steps so far while
 *                 t < window - 1), with the variability pre-activation
 *                 x = (I0 lambda)(mean + delta); the mean is
 *                 (float)sum / (float)count, each rounded once.  A job keeps
 *                 the window on the device (4 window bytes per p-bit and
 *                 trial). */
#define PSA_ALG_PSA 0u
#define PSA_ALG_SPSA 1u
#define PSA_ALG_TAPSA 2u

/* Field-computation path of a run (psa_run_desc.flags).  AUTO picks by a
 * cost model (long rows -> dense); CSR walks the sparse rows from LDS /
 * L2; DENSE multiplies the dense coupling matrix with the spins of all
 * trials on the int8 matrix cores.  The dense matrix is stored as 2-bit
 * fields times one scale when every stored coupling has the same magnitude
 * (unit and +-1 weights), else as int8 (every |J_ij| <= 127; EUNSUPPORTED
 * otherwise).  Results are identical on every path. */
#define PSA_PATH_AUTO 0u
#define PSA_PATH_CSR 1u
#define PSA_PATH_DENSE 2u
#define PSA_PATH_MASK 3u
/* With PSA_PATH_AUTO: take path and launch shape from the context's tuning
 * cache, measuring them with psa_autotune on a miss (alone for
 * psa_job_create / psa_anneal, batched inside psa_anneal_batch and the
 * server).  Launch shape never changes results. */
#define PSA_TUNE 4u

/* Fill *d with the defaults: steps 1000, trials 1, seed 0, the paper's I0
 * endpoints (i0_min = i0_max = -1), no variability (sigmas 0, p_mean 1),
 * no explicit arrays, automatic block size, plain pSA (p_stall 0.5 and
 * window 4, the paper's values, used only by SpSA and TApSA). */
void psa_run_desc_default(psa_run_desc *d);

/* Output placement flags of the read calls and psa_anneal. */
#define PSA_OUT_HOST 0u
#define PSA_OUT_DEVICE 1u

/* Create a job: upload the schedule and variability arrays, allocate the
 * device spin state (int8, [n][trials rounded up to 4], trials innermost)
 * and set the initial spins (m_i = +1 iff bit 31 of the Philox word of
 * counter (0, i/4, k, 0), word i mod 4).  The job is at step 0.
 * EUNSUPPORTED if the spin state of one workgroup's trials does not fit in
 * LDS (n above about 20,000 with 4 trials per workgroup, 80,000 with 1). */
psa_status psa_job_create(psa_ctx *ctx, const psa_graph *g,
                          const psa_run_desc *desc, psa_job **out);

/* Re-initialise the spins of every trial (as at creation) and return to
 * step 0, on the context's stream; schedule and variability are kept. */
psa_status psa_job_reset(psa_job *job);

/* Queue `k` more steps (t .. t+k-1, clipped to the schedule length) on the
 * context's stream; returns once they are queued. */
psa_status psa_job_step(psa_job *job, int32_t k);

/* How a job runs (chosen at creation). */
typedef struct psa_job_info {
    uint32_t path;             /* PSA_PATH_CSR or PSA_PATH_DENSE              */
    int32_t trials_per_group;  /* CSR: trials per workgroup (1 or 4)          */
    int32_t lanes_per_task;    /* CSR, one trial per workgroup: 1, 2 or 4     */
    int32_t block;             /* CSR: threads per workgroup                  */
    int32_t dense_encoding;    /* dense: 1 = int8 entries, 2 = 2-bit fields,
                                  3 = 1-bit fields (one coupling value)       */
    uint32_t algorithm;        /* PSA_ALG_*                                   */
    int64_t device_bytes;      /* device memory the job holds (run arrays,
                                  spin state, input-stage state, staging);
                                  its graph's is counted by the graph       */
    int32_t period_classes;    /* period mode on the class sweep: distinct
                                  periods (1..64; the sub-steps visit only
                                  the p-bits that fire); 0 otherwise        */
    int32_t period_resident;   /* with period_classes > 0: p-bits each lane
                                  keeps resident (1, 2, 4 or 8; graphs of up
                                  to 2,048 p-bits with |J| < 2^15), 0 if the
                                  sweep visits them from records            */
} psa_job_info;

psa_status psa_job_get_info(const psa_job *job, psa_job_info *out);

/* Current step index t (the number of steps applied so far). */
psa_status psa_job_position(const psa_job *job, int32_t *t);

/* Spins as int8 [trials][n] into host or device memory (flags).  Host
 * outputs synchronise the stream first. */
psa_status psa_job_read_spins(psa_job *job, int8_t *out, uint32_t flags);

/* Replace the spins of all trials by in[trials][n] (+1/-1 only; host or
 * device per flags) and set the step index to t (checkpoint / resume).
 * EUNSUPPORTED for an SpSA or TApSA job with t > 0 (its held inputs or field
 * window are not part of the spins). */
psa_status psa_job_write_spins(psa_job *job, const int8_t *in, int32_t t,
                               uint32_t flags);

/* Local fields L_i = h_i + sum_j J_ij m_j of the current spins (Eq. 3
 * without the I0 factor), int32 [trials][n]. */
psa_status psa_job_local_field(psa_job *job, int32_t *out, uint32_t flags);

/* Energy H (Eq. 2) and cut sum_{i<j} w_ij [m_i != m_j] (w = -J) of the
 * current spins, int64 [trials] each. */
psa_status psa_job_energy_cut(psa_job *job, int64_t *energy, int64_t *cut,
                              uint32_t flags);

/* psa_job_energy_cut of `count` jobs of ctx (Eq. 2 energy and cut of each
 * job's current spins) in two launches on the context's stream instead of
 * two per job, so that many small read-outs fill the device together.
 * energy[j], cut[j]: int64 [trials of jobs[j]], all host or all device
 * memory per flags (PSA_OUT_DEVICE: written in stream order, no wait; host:
 * returns when written).  Values identical to psa_job_energy_cut's.  A job
 * may be listed more than once.  EINVAL for a NULL job or output, a job of
 * another context, or more than 2^31 - 1 partial-sum workgroups or trials in
 * total; ENOMEM when a job's read-out staging cannot be allocated. */
psa_status psa_jobs_energy_cut(psa_ctx *ctx, int32_t count, psa_job *const *jobs,
                               int64_t *const *energy, int64_t *const *cut, uint32_t flags);

void psa_job_destroy(psa_job *job);

/* Whole anneal: create, all steps, energy and cut, read-out.  spins_out
 * ([trials][n]) may be NULL.  Blocks until the results are written. */
psa_status psa_anneal(psa_ctx *ctx, const psa_graph *g,
                      const psa_run_desc *desc, int8_t *spins_out,
                      int64_t *energy_out, int64_t *cut_out, uint32_t flags);

/* ------------------------------------------------------------------ */
/* Anneal without device allocation                                     */
/* ------------------------------------------------------------------ */

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it.  The same anneal as psa_anneal (identical spins, energies and
 * cuts) with every piece of run state the library needs beyond the graph
 * and the outputs -- schedule and factors as the kernels read them, spin
 * state, task order, SpSA held inputs or TApSA windows, energy partial sums
 * -- placed in one static device array of PSA_NOALLOC_SCRATCH_BYTES per
 * GPU, which the library holds from the first context on that GPU until the
 * process ends.  No hipMalloc, hipFree or other allocating call is made.
 *   - Outputs are device pointers on ctx's device: energy_out and cut_out
 *     [trials] int64 (required), spins_out [trials][n] int8 or NULL.
 *   - Sweep path only: PSA_PATH_AUTO runs the CSR sweep; PSA_PATH_DENSE
 *     gives PSA_EUNSUPPORTED (the dense path builds a coupling matrix);
 *     PSA_TUNE gives PSA_EINVAL (tuning times scratch runs); a run too large
 *     for the LDS-resident sweep gives PSA_EUNSUPPORTED.
 *   - A run whose state exceeds PSA_NOALLOC_SCRATCH_BYTES gives PSA_ENOMEM
 *     before any device work is queued, with the bytes it would need in
 *     psa_last_error().  The state is about n * trials bytes of spins plus
 *     16 n + 4 steps bytes, times 5 with SpSA and 4 window + 1 with TApSA.
 *   - Blocks until the outputs are written.  Every call on a GPU shares that
 *     GPU's array: calls that overlap on one GPU (from several threads or
 *     contexts) race and give wrong results; serialise them. */
#define PSA_NOALLOC_SCRATCH_BYTES (((size_t)128) << 20)

psa_status psa_anneal_noalloc(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                              int8_t *spins_out, int64_t *energy_out, int64_t *cut_out);

/* ------------------------------------------------------------------ */
/* Batched runs: many graphs of uneven size in one launch              */
/* ------------------------------------------------------------------ */

/* Advance every job of `jobs` (all created on ctx, each listed once) by up
 * to k steps, clipped to each job's schedule, with one launch of the batch
 * kernel on the context's stream: one work item per (job, trial) -- or per
 * (job, group of four trials) for jobs created with trials_per_group 4 --
 * each workgroup dispatching to the kernel variant its job needs.  Jobs on
 * the dense path advance on a second stream (launched step by step, a second
 * coupling encoding's jobs on a third stream beside it), joined before
 * return.  The results are identical to stepping each job alone. */
psa_status psa_jobs_step_batch(psa_ctx *ctx, int32_t count, psa_job *const *jobs,
                               int32_t k);

/* One anneal of a batch: graph, run description, and where its results go
 * (host or device memory per the flags of psa_anneal_batch). */
typedef struct psa_batch_item {
    const psa_graph *graph;
    psa_run_desc desc;
    int64_t *energy_out; /* [trials] */
    int64_t *cut_out;    /* [trials] */
    int8_t *spins_out;   /* [trials][n], or NULL */
} psa_batch_item;

/* Run the items one after the other instead of in one launch (reference). */
#define PSA_BATCH_SEQUENTIAL 2u

/* Run every item to the end of its schedule -- by default all in one
 * batched launch -- and write energies, cuts and (optionally) spins.
 * flags: PSA_OUT_HOST or PSA_OUT_DEVICE, optionally | PSA_BATCH_SEQUENTIAL.
 * Blocks until the results are written. */
psa_status psa_anneal_batch(psa_ctx *ctx, int32_t count,
                            const psa_batch_item *items, uint32_t flags);

/* ------------------------------------------------------------------ */
/* Autotuning (measured choice of path and launch shape)                 */
/* ------------------------------------------------------------------ */

/* What to tune for: one run alone (latency of its steps), or a run inside
 * batched launches (device time per run and step while other runs fill the
 * chip; timed on enough copies of the run to fill it). */
#define PSA_TUNE_ALONE 0u
#define PSA_TUNE_BATCH 1u

typedef struct psa_tune_result {
    uint32_t path;             /* PSA_PATH_CSR or PSA_PATH_DENSE            */
    int32_t trials_per_group;  /* CSR alone: 1 or 4; 0 = automatic          */
    int32_t lanes_per_task;    /* CSR: 1, 2 or 4; 0 = automatic              */
    int32_t candidates;        /* configurations timed                      */
    double us_per_step;        /* best measured, microseconds per run-step  */
    double csr_us_per_step;    /* best CSR configuration (< 0: none ran)    */
    double dense_us_per_step;  /* dense path (< 0: not applicable)          */
    double model_csr_us;       /* the cost model's estimates, for reference */
    double model_dense_us;     /* (< 0: not applicable)                     */
} psa_tune_result;

/* Time every applicable configuration -- CSR with one trial per workgroup
 * at 1, 2 or 4 lanes per task (2 or 4 when batched), CSR with four trials
 * per workgroup, and the dense path when the couplings have a dense
 * encoding -- on
 * scratch runs of `desc` (same graph, trials, schedule and factors) over
 * `probe_steps` steps (>= 1, clipped to the schedule) after one warm-up
 * step, and return the fastest.  The result is also stored in the
 * context's tuning cache, keyed by mode, trials (in batched mode, trials
 * within a half octave), update rule and the graph's shape class (n and
 * mean degree within about 9 % and 19 %, coupling encoding, rows of at most
 * 255 entries), for PSA_TUNE.  Queues and waits on the context's stream;
 * the caller's jobs are not touched. */
psa_status psa_autotune(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                        int32_t probe_steps, uint32_t mode, psa_tune_result *out);

/* The tuning cache's entry for (g, desc->trials, mode); on a miss,
 * psa_autotune with 8 probe steps (which stores it). */
psa_status psa_tune_get(psa_ctx *ctx, const psa_graph *g, const psa_run_desc *desc,
                        uint32_t mode, psa_tune_result *out);

/* Copy a tuning result's path and launch shape into a run description. */
void psa_tune_apply(const psa_tune_result *r, psa_run_desc *desc);

/* Entries in the context's tuning cache; psa_tune_clear empties it. */
int32_t psa_tune_cache_size(psa_ctx *ctx);
void psa_tune_clear(psa_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Serving with continuous batching                                     */
/* ------------------------------------------------------------------ */

typedef struct psa_server psa_server;

/* Admission limits.  hbm_budget_bytes <= 0: half of the device memory free
 * at creation; max_resident <= 0: 64 jobs; quantum_steps <= 0: 250;
 * max_waiting <= 0: no limit on jobs queued but not yet resident (else
 * psa_server_submit returns PSA_EAGAIN while that many wait). */
typedef struct psa_server_opts {
    int64_t hbm_budget_bytes; /* device bytes resident jobs may hold       */
    int32_t max_resident;     /* jobs advanced together in one launch      */
    int32_t quantum_steps;    /* steps per launch between scheduling points */
    int32_t max_waiting;      /* queued jobs accepted before PSA_EAGAIN    */
} psa_server_opts;

/* Job states. */
#define PSA_JOB_QUEUED 0
#define PSA_JOB_RUNNING 1
#define PSA_JOB_DONE 2
#define PSA_JOB_ERROR 3
#define PSA_JOB_CANCELED 4

typedef struct psa_result {
    int32_t status;    /* PSA_JOB_*                                      */
    int32_t error;     /* psa_status of a failed job (PSA_OK otherwise)  */
    int64_t submit_us; /* times in microseconds since server creation   */
    int64_t admit_us;  /* -1 until admitted (device memory reserved)     */
    int64_t start_us;  /* -1 until its first step quantum is launched    */
    int64_t end_us;    /* -1 until done, failed or canceled              */
} psa_result;

typedef struct psa_server_stats {
    int32_t waiting, resident;
    int64_t completed, failed, canceled, quanta;
    int64_t used_bytes, budget_bytes;
    int32_t peak_resident;   /* most jobs resident at once so far       */
    int64_t peak_used_bytes; /* most device bytes held at once so far   */
} psa_server_stats;

/* Start a server on ctx.  Its scheduler thread issues all device work on the
 * context's stream from then on: do not use ctx from other threads while the
 * server exists.  Between step quanta it retires finished jobs, admits
 * waiting jobs first come first served while their device footprint fits
 * the budget and a slot is free, and advances every resident job by one
 * quantum in a single batched launch (psa_jobs_step_batch).  A job's results
 * are identical to running it alone.
 * Footprint: admission reserves an estimate of what the job will hold (its
 * graph in every encoding, the dense coupling matrix and dense spin buffers
 * when the dense path may be chosen, the run state, read-out staging, and
 * the scratch runs the autotuner times with PSA_TUNE); once the job is
 * created the reservation is replaced by the device bytes it actually holds
 * (graph and job, psa_graph_info.device_bytes + psa_job_info.device_bytes),
 * and a dense matrix the chosen path does not read is freed. */
psa_status psa_server_create(psa_ctx *ctx, const psa_server_opts *opts,
                             psa_server **out);

/* Queue one anneal: a graph as an edge list (as psa_graph_from_edges; the
 * arrays are copied) and a run description (its optional arrays are
 * copied).  energy_out / cut_out ([trials]) and spins_out ([trials][n] or
 * NULL) are host buffers the server fills when the job is done; they must
 * stay valid until the job reports DONE, ERROR or CANCELED.  A job whose
 * footprint alone exceeds the budget ends in ERROR with PSA_ENOMEM.
 * PSA_EAGAIN (nothing queued, *ticket untouched) while max_waiting jobs
 * wait for admission. */
psa_status psa_server_submit(psa_server *s, int32_t n, int64_t m,
                             const int32_t *u, const int32_t *v,
                             const int32_t *val, const int32_t *h,
                             uint32_t graph_flags, const psa_run_desc *desc,
                             int64_t *energy_out, int64_t *cut_out,
                             int8_t *spins_out, uint64_t *ticket);

/* Current state of a job (never blocks). */
psa_status psa_server_poll(psa_server *s, uint64_t ticket, psa_result *out);

/* Block until the job is done, failed or canceled, or timeout_us passes
 * (timeout_us < 0: no limit; PSA_ETIMEDOUT with the current state). */
psa_status psa_server_wait(psa_server *s, uint64_t ticket, int64_t timeout_us,
                           psa_result *out);

/* Ask for a job to be dropped (queued: at once; resident: after the current
 * quantum).  A job that has already finished keeps its results. */
psa_status psa_server_cancel(psa_server *s, uint64_t ticket);

/* Forget a finished job's record (its ticket becomes unknown). */
psa_status psa_server_release(psa_server *s, uint64_t ticket);

psa_status psa_server_stats_get(psa_server *s, psa_server_stats *out);

/* Stop the server: queued jobs are canceled, resident jobs are canceled
 * after the current quantum, the scheduler thread is joined. */
void psa_server_destroy(psa_server *s);

/* ------------------------------------------------------------------ */
/* Value-level checks of the per-update arithmetic (tests)              */
/* ------------------------------------------------------------------ */

/* y[i] = the device's single-precision tanh of x[i] (Eq. 1's activation;
 * the operation order is fixed: tanh(x) = sign(x) (1 - 2/(2^v + 1)) with
 * v = |x| RN(2 log2 e), 2^v from a degree-7 Taylor polynomial of 2^f and an
 * exact scaling, a correctly rounded division, |x| >= 9 giving +-1).
 * x and y are device pointers to count floats; asynchronous on the
 * context's stream. */
psa_status psa_debug_tanh(psa_ctx *ctx, int64_t count, const float *x, float *y);

/* out[i] = the decision the kernels take for an input x[i] and the random
 * word rword[i] of the r stream (Eq. 1: +1 iff tanh(x) > r, r the odd
 * multiple of 2^-24 given by the top 24 bits of the word): bit 0 is set for
 * +1; bit 1 is set when the hardware estimate of tanh lay within 2^-16 of r,
 * so that the exact tanh of psa_debug_tanh decided.  Device pointers to
 * count elements; asynchronous on the context's stream. */
psa_status psa_debug_decide(psa_ctx *ctx, int64_t count, const float *x, const uint32_t *rword,
                            uint8_t *out);

/* The bound of one dependency wait of the persistent dense launch
 * (PSA_DENSE_LAUNCH_PERSISTENT), in polls of the run's counter: 2^20 by
 * default (about a second).  A test entry for the failure path: with 0
 * every wait of a quantum of two or more steps gives up at once, the
 * workgroups leave normally, and the next dense quantum on the context
 * returns PSA_EHIP.  EINVAL: ctx NULL. */
psa_status psa_debug_dense_wait_limit(psa_ctx *ctx, uint32_t max_polls);

#ifdef __cplusplus
}
#endif

#endif /* PSA_H */
