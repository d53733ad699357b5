/*
 * psa_oracle.h -- declarations of the reference (oracle) implementation of
 * p-bit simulated annealing (pSA) with device variability.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and psa_oracle.c are a plain,
 * slow, single-threaded C restatement of the method of Onizawa & Hanyu,
 * "GPU-accelerated simulated annealing based on p-bits with real-world
 * device-variability modeling" (arXiv 2601.14476).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library, and the
 * GPU library never calls it.
 *
 * Conventions shared by every entry point:
 *   - Graphs are undirected edge lists (eu[e], ev[e], ej[e]) of Ising
 *     couplings J_{uv} = ej[e] (Eq. 2), each unordered pair listed once,
 *     no self loops, plus an optional bias vector h (NULL = all zero).
 *   - Spins are int8 in {-1,+1}, stored trial-major: spins[k*n + i] is
 *     p-bit i of trial k, for the trials [trial_begin, trial_end) of the
 *     call, local row index k - trial_begin.
 *   - Return value 0 = success, -1 = invalid argument, -2 = out of memory.
 */
#ifndef PSA_ORACLE_H
#define PSA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block: out = Philox(ctr, key). */
void psa_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                           uint32_t out[4]);

/* The 32-bit random word that p-bit i of trial k draws at step t for the
 * purpose `tag` (0 = initial spin, 1 = r, 2 = timing gate): word i mod 4 of
 * the Philox block of counter (t, i/4, k, tag). */
uint32_t psa_ref_word(uint64_t seed, uint32_t t, uint32_t i, uint32_t k,
                      uint32_t tag);

/* Uniform r in (-1,1) from a random word (Eq. 1). */
float psa_ref_r_from_word(uint32_t u);

/* Timing gate: 1 if the p-bit updates this step. */
int psa_ref_gate(uint32_t u, uint32_t thr24);

/* tanh in single precision, evaluated by a fixed operation sequence. */
float psa_ref_tanh(float x);

/* Element-wise tanh and r maps over `count` values (exhaustive tests). */
void psa_ref_tanh_array(int64_t count, const float *x, float *y);
void psa_ref_r_array(int64_t count, const uint32_t *u, float *r);

/* Paper schedule endpoints: mean(s_i) over the dense coupling rows. */
int psa_ref_mean_s(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   const int32_t *ej, double *mean_s);

/* Geometric I0 schedule, I0(t+1) = I0(t) / beta. */
int psa_ref_schedule(int32_t steps, double i0_min, double i0_max,
                     float *i0_out);

/* Device-variability draw (Eq. 7): lambda_i, delta_i and the per-step
 * update probability of the timing factor, quantised to thr24_i. */
int psa_ref_variability(int32_t n, uint64_t seed, double sigma_lambda,
                        double sigma_delta, double sigma_nu, double p_mean,
                        float *lambda_out, float *offset_out,
                        uint32_t *thr24_out);

/* Initial spins of trials [trial_begin, trial_end). */
int psa_ref_init_spins(int32_t n, uint64_t seed, int32_t trial_begin,
                       int32_t trial_end, int8_t *spins);

/* Local fields L_i = h_i + sum_j J_ij m_j (Eq. 3 without I0) for each
 * trial row of `spins`; out has the same [rows][n] layout, int32. */
int psa_ref_local_field(int32_t n, int64_t m, const int32_t *eu,
                        const int32_t *ev, const int32_t *ej,
                        const int32_t *h, int32_t rows, const int8_t *spins,
                        int32_t *out);

/* Run the synchronous p-bit sweeps t = t_begin .. t_end-1 on the trials
 * [trial_begin, trial_end), spins updated in place.  i0 holds the whole
 * schedule (index t); lambda/offset/thr24 are per p-bit. */
int psa_ref_run(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                const int32_t *ej, const int32_t *h, const float *i0,
                const float *lambda, const float *offset,
                const uint32_t *thr24, uint64_t seed, int32_t trial_begin,
                int32_t trial_end, int32_t t_begin, int32_t t_end,
                int8_t *spins);

/* Stalled-input variant (SpSA, Eq. 5): the input of a p-bit keeps its
 * previous value with probability stall24 / 2^24, else it is formed anew
 * from the spins of step t; the output rule (gate, r, tanh) is the pSA one.
 * The held input is the whole pre-activation x_i of the last refresh (I0
 * and the variability factors of that step included).  Step 0 always
 * refreshes.  x_state ([trials][n] floats, same rows as spins) carries the
 * inputs between calls: read when t_begin > 0, written on return.
 * Randomness: the stall word is Philox word i mod 4 of counter
 * (t, i/4, k, 4); the input stalls iff (word >> 8) < stall24. */
int psa_ref_run_spsa(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     const int32_t *ej, const int32_t *h, const float *i0,
                     const float *lambda, const float *offset,
                     const uint32_t *thr24, uint32_t stall24, uint64_t seed,
                     int32_t trial_begin, int32_t trial_end, int32_t t_begin,
                     int32_t t_end, int8_t *spins, float *x_state);

/* Time-averaged variant (TApSA, Eq. 4): the input of a p-bit is I0 times
 * the mean of its last alpha fields TI(t) = h + sum_j J m_j(t) (the
 * available ones while t < alpha - 1), here with the device-variability
 * pre-activation x = (I0 lambda_i)(mean + delta_i), the mean computed as
 * (float)sum / (float)count, each rounded once.  ring ([trials][n][alpha]
 * int32, same rows as spins) holds the window: field of step t in slot
 * t mod alpha; read when t_begin > 0, written on return. */
int psa_ref_run_tapsa(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                      const int32_t *ej, const int32_t *h, const float *i0,
                      const float *lambda, const float *offset,
                      const uint32_t *thr24, int32_t alpha, uint64_t seed,
                      int32_t trial_begin, int32_t trial_end, int32_t t_begin,
                      int32_t t_end, int8_t *spins, int32_t *ring);

/* Ising energy (Eq. 2) and cut weight with w = -J of each trial row. */
int psa_ref_energy_cut(int32_t n, int64_t m, const int32_t *eu,
                       const int32_t *ev, const int32_t *ej, const int32_t *h,
                       int32_t rows, const int8_t *spins, int64_t *energy,
                       int64_t *cut);

/* Whole anneal: initial spins, steps 0..steps-1, final energy and cut. */
int psa_ref_anneal(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   const int32_t *ej, const int32_t *h, int32_t steps,
                   const float *i0, const float *lambda, const float *offset,
                   const uint32_t *thr24, uint64_t seed, int32_t trial_begin,
                   int32_t trial_end, int8_t *spins, int64_t *energy,
                   int64_t *cut);

#ifdef __cplusplus
}
#endif

#endif /* PSA_ORACLE_H */
