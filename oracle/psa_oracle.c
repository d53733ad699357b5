/*
 * psa_oracle.c -- reference (oracle) implementation of p-bit simulated
 * annealing with device variability, after Onizawa & Hanyu,
 * "GPU-accelerated simulated annealing based on p-bits with real-world
 * device-variability modeling" (arXiv 2601.14476).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It is kept
 * plain on purpose -- one trial at a time, one p-bit at a time, one Philox
 * block per random word -- so that it can be checked against the paper by
 * eye.  It shares no code with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared psa_oracle.c -lm
 * (no fast-math, no contraction: the single-precision operations below are
 * each rounded exactly once, in the order written).
 *
 * Readings of the paper taken here (each one is also listed with its
 * reason in the design notes of the repository):
 *   - update rule: Eq. 1 / Eq. 6 and the pseudo-code listing of the
 *     SimulatedAnnealingModule; all p-bits of a step read the spins of the
 *     previous step (synchronous update, as the Introduction and the
 *     Discussion describe it);  m = +1 iff tanh(x) > r, ties give -1;
 *   - pre-activation x = (I0 * lambda_i) * ((float)L_i + delta_i), with
 *     L_i = h_i + sum_j J_ij m_j, i.e. the offset is added to the integer
 *     field before the I0 scaling, as in the listing;
 *   - timing variability (nu, Eq. 6/7) is modelled as a per-p-bit update
 *     probability p_i drawn once per run; a p-bit that does not fire in a
 *     step keeps its output;
 *   - r is uniform on the odd multiples of 2^-24 in (-1,1);
 *   - randomness: Philox4x32-10 with key = seed and counter
 *     (step, p-bit/4, trial, purpose); p-bit i uses word i mod 4.
 *   - schedule: I0(t+1) = I0(t)/beta, beta = (I0min/I0max)^(1/(S-1)),
 *     computed in double and rounded to float per step;
 *   - I0min = 0.1/mean(s), I0max = 10/mean(s), s_i = sqrt((n-1) Var(J_i,:))
 *     with the population variance over the whole dense row (n entries).
 */
#include "psa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TAG_INIT 0u
#define TAG_R 1u
#define TAG_GATE 2u
#define TAG_VAR 3u
#define TAG_STALL 4u

#define GATE_ONE (1u << 24)

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  A round maps  */
/* (c0,c1,c2,c3) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1,     */
/* lo(M0*c0)); the key is bumped by the Weyl constants between rounds. */
/* ------------------------------------------------------------------ */
void psa_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                           uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Fresh randomness per (step, p-bit, trial): the listing draws a new
 * random vector rnd every cycle.  Counter = (t, i/4, k, tag): one block
 * serves the four p-bits 4(i/4) .. 4(i/4)+3 of trial k, word i%4. */
uint32_t psa_ref_word(uint64_t seed, uint32_t t, uint32_t i, uint32_t k,
                      uint32_t tag)
{
    uint32_t ctr[4] = {t, i >> 2, k, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    psa_ref_philox4x32_10(ctr, key, out);
    return out[i & 3u];
}

/* Eq. 1: r_i(t) uniform in (-1,1).  The top 25 bits with the lowest bit
 * forced to one give an odd integer j in [1, 2^25); r = (j - 2^24)/2^24
 * is then an odd multiple of 2^-24, exactly representable, never zero,
 * and symmetric about zero. */
float psa_ref_r_from_word(uint32_t u)
{
    int32_t j = (int32_t)((u >> 7) | 1u);
    return (float)(j - (int32_t)GATE_ONE) * 0x1p-24f;
}

/* Timing factor: the p-bit fires with probability thr24 / 2^24. */
int psa_ref_gate(uint32_t u, uint32_t thr24)
{
    if (thr24 >= GATE_ONE)
        return 1;
    return (u >> 8) < thr24;
}

/* tanh(x) = sign(x) * (1 - 2/(e^{2|x|} + 1)).  e^{2|x|} = 2^v with
 * v = 2|x| log2(e); v = n + f with n the nearest integer and |f| <= 1/2;
 * 2^f = e^{f ln 2} by its Taylor series sum_k (ln 2)^k f^k / k! to degree
 * 7 (Horner, fused multiply-adds); the coefficients are (ln 2)^k / k!
 * rounded to float.  For |x| >= 9 the value is 1 (tanh(9) is within
 * 2^-24 of one). */
float psa_ref_tanh(float x)
{
    float a = fabsf(x);
    float y;
    if (a >= 9.0f) {
        y = 1.0f;
    } else {
        float v = a * 0x1.715476p+1f; /* 2 log2(e) */
        float nf = rintf(v);
        float f = v - nf;
        float p = 0x1.ffcbfcp-17f;    /* (ln2)^7 / 7! */
        p = fmaf(p, f, 0x1.430912p-13f); /* (ln2)^6 / 6! */
        p = fmaf(p, f, 0x1.5d87fep-10f); /* (ln2)^5 / 5! */
        p = fmaf(p, f, 0x1.3b2ab6p-7f);  /* (ln2)^4 / 4! */
        p = fmaf(p, f, 0x1.c6b08ep-5f);  /* (ln2)^3 / 3! */
        p = fmaf(p, f, 0x1.ebfbe0p-3f);  /* (ln2)^2 / 2! */
        p = fmaf(p, f, 0x1.62e430p-1f);  /* ln2 */
        p = fmaf(p, f, 1.0f);
        float e = ldexpf(p, (int)nf);    /* e^{2|x|} */
        y = 1.0f - 2.0f / (e + 1.0f);
    }
    return copysignf(y, x);
}

/* Element-wise versions for exhaustive tests of the three maps above. */
void psa_ref_tanh_array(int64_t count, const float *x, float *y)
{
    for (int64_t q = 0; q < count; q++)
        y[q] = psa_ref_tanh(x[q]);
}

void psa_ref_r_array(int64_t count, const uint32_t *u, float *r)
{
    for (int64_t q = 0; q < count; q++)
        r[q] = psa_ref_r_from_word(u[q]);
}

/* ------------------------------------------------------------------ */
/* Graph handling: plain adjacency lists built from the edge list.     */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t *start; /* [n+1] */
    int32_t *nbr;   /* [2m] */
    int32_t *w;     /* [2m] coupling J_ij */
} ref_adj;

static void adj_free(ref_adj *a)
{
    free(a->start);
    free(a->nbr);
    free(a->w);
}

static int cmp_pair(const void *pa, const void *pb)
{
    const int64_t x = *(const int64_t *)pa, y = *(const int64_t *)pb;
    return (x > y) - (x < y);
}

/* Validates the edge list (indices in range, no self loop, no repeated
 * pair, |field| < 2^24 so that (float)L is exact) and builds adjacency. */
static int adj_build(int32_t n, int64_t m, const int32_t *eu,
                     const int32_t *ev, const int32_t *ej, const int32_t *h,
                     ref_adj *a)
{
    memset(a, 0, sizeof(*a));
    if (n < 1 || m < 0 || (m > 0 && (!eu || !ev || !ej)))
        return -1;
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *absrow = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    a->start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    a->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    a->w = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    if (!keys || !absrow || !a->start || !a->nbr || !a->w) {
        free(keys);
        free(absrow);
        adj_free(a);
        return -2;
    }
    int rc = 0;
    for (int64_t e = 0; e < m && rc == 0; e++) {
        int32_t u = eu[e], v = ev[e];
        if (u < 0 || u >= n || v < 0 || v >= n || u == v) {
            rc = -1;
            break;
        }
        int32_t lo = u < v ? u : v, hi = u < v ? v : u;
        keys[e] = (int64_t)lo * (int64_t)n + hi;
        int64_t aw = ej[e] < 0 ? -(int64_t)ej[e] : (int64_t)ej[e];
        absrow[u] += aw;
        absrow[v] += aw;
        a->start[u + 1]++;
        a->start[v + 1]++;
    }
    if (rc == 0 && m > 1) {
        qsort(keys, (size_t)m, sizeof(int64_t), cmp_pair);
        for (int64_t e = 1; e < m; e++)
            if (keys[e] == keys[e - 1])
                rc = -1;
    }
    for (int32_t i = 0; i < n && rc == 0; i++) {
        int64_t hb = h ? (h[i] < 0 ? -(int64_t)h[i] : (int64_t)h[i]) : 0;
        if (hb + absrow[i] >= (int64_t)GATE_ONE)
            rc = -1;
    }
    free(keys);
    free(absrow);
    if (rc != 0) {
        adj_free(a);
        return rc;
    }
    a->n = n;
    for (int32_t i = 0; i < n; i++)
        a->start[i + 1] += a->start[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!fill) {
        adj_free(a);
        return -2;
    }
    for (int32_t i = 0; i < n; i++)
        fill[i] = a->start[i];
    for (int64_t e = 0; e < m; e++) {
        int32_t u = eu[e], v = ev[e];
        a->nbr[fill[u]] = v;
        a->w[fill[u]++] = ej[e];
        a->nbr[fill[v]] = u;
        a->w[fill[v]++] = ej[e];
    }
    free(fill);
    return 0;
}

/* Eq. 3 without the I0 factor: L_i = h_i + sum_j J_ij m_j. */
static int32_t field_of(const ref_adj *a, const int32_t *h, int32_t i,
                        const int8_t *m)
{
    int32_t L = h ? h[i] : 0;
    for (int64_t p = a->start[i]; p < a->start[i + 1]; p++)
        L += a->w[p] * (int32_t)m[a->nbr[p]];
    return L;
}

/* ------------------------------------------------------------------ */
/* Schedule (Methods, experimental conditions).                        */
/* ------------------------------------------------------------------ */
int psa_ref_mean_s(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   const int32_t *ej, double *mean_s)
{
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, NULL, &a);
    if (rc != 0)
        return rc;
    if (!mean_s) {
        adj_free(&a);
        return -1;
    }
    /* Var over the n entries of the dense row J_{i,:} (zeros included):
     * Var = (n*sum J^2 - (sum J)^2) / n^2, numerator exact in int64. */
    double sum = 0.0;
    for (int32_t i = 0; i < n; i++) {
        int64_t s1 = 0, s2 = 0;
        for (int64_t p = a.start[i]; p < a.start[i + 1]; p++) {
            s1 += a.w[p];
            s2 += (int64_t)a.w[p] * (int64_t)a.w[p];
        }
        int64_t num = (int64_t)n * s2 - s1 * s1;
        double var = (double)num / ((double)n * (double)n);
        double s = sqrt((double)(n - 1) * var);
        sum += s;
    }
    *mean_s = sum / (double)n;
    adj_free(&a);
    return 0;
}

int psa_ref_schedule(int32_t steps, double i0_min, double i0_max,
                     float *i0_out)
{
    if (steps < 1 || !i0_out || !(i0_min > 0.0) || !(i0_max >= i0_min))
        return -1;
    if (steps == 1) {
        i0_out[0] = (float)i0_min;
        return 0;
    }
    double beta = pow(i0_min / i0_max, 1.0 / (double)(steps - 1));
    double I0 = i0_min;
    for (int32_t t = 0; t < steps; t++) {
        i0_out[t] = (float)I0;
        I0 = I0 / beta;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. 7: lambda ~ N(1, s_l^2), delta ~ N(0, s_d^2), and the timing     */
/* factor as an update probability p ~ clip(N(p_mean, s_n^2), 0, 1).    */
/* Normals by the Box-Muller transform (cosine branch only), one pair  */
/* of Philox words per normal.                                         */
/* ------------------------------------------------------------------ */
static double box_muller_cos(uint32_t w1, uint32_t w2)
{
    double u1 = ((double)w1 + 1.0) / 4294967296.0; /* (0,1] */
    double u2 = (double)w2 / 4294967296.0;         /* [0,1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

int psa_ref_variability(int32_t n, uint64_t seed, double sigma_lambda,
                        double sigma_delta, double sigma_nu, double p_mean,
                        float *lambda_out, float *offset_out,
                        uint32_t *thr24_out)
{
    if (n < 1 || !lambda_out || !offset_out || !thr24_out)
        return -1;
    if (!(sigma_lambda >= 0.0) || !(sigma_delta >= 0.0) || !(sigma_nu >= 0.0) ||
        !(p_mean >= 0.0 && p_mean <= 1.0))
        return -1;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int32_t i = 0; i < n; i++) {
        uint32_t c0[4] = {0u, (uint32_t)i, 0u, TAG_VAR};
        uint32_t c1[4] = {0u, (uint32_t)i, 1u, TAG_VAR};
        uint32_t w[4], x[4];
        psa_ref_philox4x32_10(c0, key, w);
        psa_ref_philox4x32_10(c1, key, x);
        double z_lambda = box_muller_cos(w[0], w[1]);
        double z_delta = box_muller_cos(w[2], w[3]);
        double z_nu = box_muller_cos(x[0], x[1]);
        lambda_out[i] = (float)(1.0 + sigma_lambda * z_lambda);
        offset_out[i] = (float)(sigma_delta * z_delta);
        double p = p_mean + sigma_nu * z_nu;
        if (p < 0.0)
            p = 0.0;
        if (p > 1.0)
            p = 1.0;
        thr24_out[i] = (uint32_t)floor(p * 16777216.0);
    }
    return 0;
}

/* Eq. 6's timing factor nu_i as the integer period of the listing's gate
 * (count mod nu[i]): the nominal period is one cycle of t_res sub-steps
 * and nu_i stretches or shortens it. */
int psa_ref_periods(int32_t n, uint64_t seed, double sigma_nu, int32_t t_res,
                    uint32_t *period_out)
{
    if (n < 1 || !period_out || t_res < 1 || !(sigma_nu >= 0.0))
        return -1;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int32_t i = 0; i < n; i++) {
        uint32_t c1[4] = {0u, (uint32_t)i, 1u, TAG_VAR};
        uint32_t x[4];
        psa_ref_philox4x32_10(c1, key, x);
        double nu = sigma_nu * box_muller_cos(x[0], x[1]);
        double p = rint((double)t_res * (1.0 + nu));
        period_out[i] = p < 1.0 ? 1u : (uint32_t)p;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Initial state: uniform +-1 from the top bit of the INIT word.        */
/* ------------------------------------------------------------------ */
int psa_ref_init_spins(int32_t n, uint64_t seed, int32_t trial_begin,
                       int32_t trial_end, int8_t *spins)
{
    if (n < 1 || trial_begin < 0 || trial_end < trial_begin || !spins)
        return -1;
    for (int32_t k = trial_begin; k < trial_end; k++) {
        int8_t *mk = spins + (int64_t)(k - trial_begin) * n;
        for (int32_t i = 0; i < n; i++) {
            uint32_t u = psa_ref_word(seed, 0u, (uint32_t)i, (uint32_t)k, TAG_INIT);
            mk[i] = (u >> 31) ? (int8_t)1 : (int8_t)-1;
        }
    }
    return 0;
}

int psa_ref_local_field(int32_t n, int64_t m, const int32_t *eu,
                        const int32_t *ev, const int32_t *ej,
                        const int32_t *h, int32_t rows, const int8_t *spins,
                        int32_t *out)
{
    if (rows < 0 || (rows > 0 && (!spins || !out)))
        return -1;
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, h, &a);
    if (rc != 0)
        return rc;
    for (int32_t k = 0; k < rows; k++)
        for (int32_t i = 0; i < n; i++)
            out[(int64_t)k * n + i] = field_of(&a, h, i, spins + (int64_t)k * n);
    adj_free(&a);
    return 0;
}

/* ------------------------------------------------------------------ */
/* pSA sweeps with the variability p-bit of Eq. 6.                      */
/* ------------------------------------------------------------------ */
int psa_ref_run(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                const int32_t *ej, const int32_t *h, const float *i0,
                const float *lambda, const float *offset,
                const uint32_t *thr24, uint64_t seed, int32_t trial_begin,
                int32_t trial_end, int32_t t_begin, int32_t t_end,
                int8_t *spins)
{
    if (!i0 || !lambda || !offset || !thr24 || !spins || trial_begin < 0 ||
        trial_end < trial_begin || t_begin < 0 || t_end < t_begin)
        return -1;
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, h, &a);
    if (rc != 0)
        return rc;
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int8_t *next = (int8_t *)malloc((size_t)n);
    if (!L || !next) {
        free(L);
        free(next);
        adj_free(&a);
        return -2;
    }
    for (int32_t k = trial_begin; k < trial_end; k++) {
        int8_t *mk = spins + (int64_t)(k - trial_begin) * n;
        for (int32_t t = t_begin; t < t_end; t++) {
            /* Every p-bit's input is formed from the outputs of step t. */
            for (int32_t i = 0; i < n; i++)
                L[i] = field_of(&a, h, i, mk);
            for (int32_t i = 0; i < n; i++) {
                uint32_t ug = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_GATE);
                if (!psa_ref_gate(ug, thr24[i])) {
                    next[i] = mk[i]; /* p-bit does not fire: output held */
                    continue;
                }
                uint32_t ur = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_R);
                float r = psa_ref_r_from_word(ur);
                float a_i = i0[t] * lambda[i];        /* I0 * lambda_i   */
                float b_i = (float)L[i] + offset[i];  /* field + delta_i */
                float x = a_i * b_i;
                float y = psa_ref_tanh(x);
                next[i] = (y > r) ? (int8_t)1 : (int8_t)-1;
            }
            memcpy(mk, next, (size_t)n);
        }
    }
    free(L);
    free(next);
    adj_free(&a);
    return 0;
}

/* SpSA (Eq. 5).  Per step and trial: every p-bit first decides whether its
 * input I_i is stalled (kept from the previous step, with probability
 * stall24 / 2^24) or formed anew, I_i = I0 (h_i + sum_j J_ij m_j(t)), here
 * with the device-variability pre-activation x = (I0 lambda_i)(L_i +
 * delta_i); then the p-bit output follows Eq. 1 / Eq. 6 with the held or
 * fresh input, under the same timing gate as pSA. */
int psa_ref_run_spsa(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     const int32_t *ej, const int32_t *h, const float *i0,
                     const float *lambda, const float *offset,
                     const uint32_t *thr24, uint32_t stall24, uint64_t seed,
                     int32_t trial_begin, int32_t trial_end, int32_t t_begin,
                     int32_t t_end, int8_t *spins, float *x_state)
{
    if (!i0 || !lambda || !offset || !thr24 || !spins || !x_state ||
        trial_begin < 0 || trial_end < trial_begin || t_begin < 0 ||
        t_end < t_begin || stall24 > GATE_ONE)
        return -1;
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, h, &a);
    if (rc != 0)
        return rc;
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int8_t *next = (int8_t *)malloc((size_t)n);
    if (!L || !next) {
        free(L);
        free(next);
        adj_free(&a);
        return -2;
    }
    for (int32_t k = trial_begin; k < trial_end; k++) {
        int8_t *mk = spins + (int64_t)(k - trial_begin) * n;
        float *xk = x_state + (int64_t)(k - trial_begin) * n;
        for (int32_t t = t_begin; t < t_end; t++) {
            for (int32_t i = 0; i < n; i++)
                L[i] = field_of(&a, h, i, mk);
            for (int32_t i = 0; i < n; i++) {
                /* input stage: held with probability p, else fresh */
                uint32_t us = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_STALL);
                int stalled = t > 0 && (us >> 8) < stall24;
                if (!stalled) {
                    float a_i = i0[t] * lambda[i];
                    float b_i = (float)L[i] + offset[i];
                    xk[i] = a_i * b_i;
                }
                /* output stage: as pSA, on the held or fresh input */
                uint32_t ug = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_GATE);
                if (!psa_ref_gate(ug, thr24[i])) {
                    next[i] = mk[i];
                    continue;
                }
                uint32_t ur = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_R);
                float r = psa_ref_r_from_word(ur);
                next[i] = (psa_ref_tanh(xk[i]) > r) ? (int8_t)1 : (int8_t)-1;
            }
            memcpy(mk, next, (size_t)n);
        }
    }
    free(L);
    free(next);
    adj_free(&a);
    return 0;
}

/* Period-mode timing (Eq. 6, listing): the simulation advances in sub-steps
 * of 1/t_res cycle; a p-bit fires at the sub-steps that are multiples of its
 * period and otherwise holds its output. */
int psa_ref_run_period(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                       const int32_t *ej, const int32_t *h, const float *i0,
                       const float *lambda, const float *offset,
                       const uint32_t *period, int32_t t_res, uint64_t seed,
                       int32_t trial_begin, int32_t trial_end, int32_t t_begin,
                       int32_t t_end, int8_t *spins)
{
    if (!i0 || !lambda || !offset || !period || !spins || t_res < 1 ||
        trial_begin < 0 || trial_end < trial_begin || t_begin < 0 || t_end < t_begin)
        return -1;
    for (int32_t i = 0; i < n; i++)
        if (period[i] < 1)
            return -1;
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, h, &a);
    if (rc != 0)
        return rc;
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int8_t *next = (int8_t *)malloc((size_t)n);
    if (!L || !next) {
        free(L);
        free(next);
        adj_free(&a);
        return -2;
    }
    for (int32_t k = trial_begin; k < trial_end; k++) {
        int8_t *mk = spins + (int64_t)(k - trial_begin) * n;
        for (int32_t t = t_begin; t < t_end; t++) {
            for (int32_t s = 0; s < t_res; s++) {
                uint32_t tau = (uint32_t)t * (uint32_t)t_res + (uint32_t)s;
                for (int32_t i = 0; i < n; i++)
                    L[i] = field_of(&a, h, i, mk);
                for (int32_t i = 0; i < n; i++) {
                    if (tau % period[i] != 0) {
                        next[i] = mk[i];
                        continue;
                    }
                    uint32_t ur = psa_ref_word(seed, tau, (uint32_t)i, (uint32_t)k, TAG_R);
                    float r = psa_ref_r_from_word(ur);
                    float a_i = i0[t] * lambda[i];
                    float b_i = (float)L[i] + offset[i];
                    float x = a_i * b_i;
                    next[i] = (psa_ref_tanh(x) > r) ? (int8_t)1 : (int8_t)-1;
                }
                memcpy(mk, next, (size_t)n);
            }
        }
    }
    free(L);
    free(next);
    adj_free(&a);
    return 0;
}

/* TApSA (Eq. 4).  Per step and trial: every p-bit forms its temporary field
 * TI_i(t) (Eq. 4a, the integer field of the spins of step t) and records it
 * in its window; its input is I0 times the mean of the window (Eq. 4b, the
 * fields of steps t, t-1, .., t-alpha+1, fewer at the start), with the
 * variability pre-activation of Eq. 6; the output follows Eq. 1 / Eq. 6. */
int psa_ref_run_tapsa(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                      const int32_t *ej, const int32_t *h, const float *i0,
                      const float *lambda, const float *offset,
                      const uint32_t *thr24, int32_t alpha, uint64_t seed,
                      int32_t trial_begin, int32_t trial_end, int32_t t_begin,
                      int32_t t_end, int8_t *spins, int32_t *ring)
{
    if (!i0 || !lambda || !offset || !thr24 || !spins || !ring || alpha < 1 ||
        trial_begin < 0 || trial_end < trial_begin || t_begin < 0 || t_end < t_begin)
        return -1;
    ref_adj a;
    int rc = adj_build(n, m, eu, ev, ej, h, &a);
    if (rc != 0)
        return rc;
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int8_t *next = (int8_t *)malloc((size_t)n);
    if (!L || !next) {
        free(L);
        free(next);
        adj_free(&a);
        return -2;
    }
    for (int32_t k = trial_begin; k < trial_end; k++) {
        int8_t *mk = spins + (int64_t)(k - trial_begin) * n;
        int32_t *rk = ring + (int64_t)(k - trial_begin) * n * alpha;
        for (int32_t t = t_begin; t < t_end; t++) {
            for (int32_t i = 0; i < n; i++)
                L[i] = field_of(&a, h, i, mk);          /* Eq. 4a */
            int32_t count = t + 1 < alpha ? t + 1 : alpha;
            for (int32_t i = 0; i < n; i++) {
                int32_t *w = rk + (int64_t)i * alpha;
                w[t % alpha] = L[i];
                int64_t sum = 0;
                for (int32_t q = 0; q < count; q++)
                    sum += w[(t - q) % alpha];
                float mean = (float)sum / (float)count;  /* Eq. 4b */
                uint32_t ug = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_GATE);
                if (!psa_ref_gate(ug, thr24[i])) {
                    next[i] = mk[i];
                    continue;
                }
                uint32_t ur = psa_ref_word(seed, (uint32_t)t, (uint32_t)i,
                                           (uint32_t)k, TAG_R);
                float r = psa_ref_r_from_word(ur);
                float a_i = i0[t] * lambda[i];
                float b_i = mean + offset[i];
                float x = a_i * b_i;
                next[i] = (psa_ref_tanh(x) > r) ? (int8_t)1 : (int8_t)-1;
            }
            memcpy(mk, next, (size_t)n);
        }
    }
    free(L);
    free(next);
    adj_free(&a);
    return 0;
}

/* Eq. 2: H = -sum_i h_i m_i - sum_{i<j} J_ij m_i m_j.  Cut of the
 * bipartition {m = +1} / {m = -1} with edge weights w = -J (the MAX-CUT
 * objective): sum over edges of w_ij [m_i != m_j]. */
int psa_ref_energy_cut(int32_t n, int64_t m, const int32_t *eu,
                       const int32_t *ev, const int32_t *ej, const int32_t *h,
                       int32_t rows, const int8_t *spins, int64_t *energy,
                       int64_t *cut)
{
    if (n < 1 || m < 0 || rows < 0 ||
        (rows > 0 && (!spins || !energy || !cut)) ||
        (m > 0 && (!eu || !ev || !ej)))
        return -1;
    for (int32_t k = 0; k < rows; k++) {
        const int8_t *mk = spins + (int64_t)k * n;
        int64_t E = 0, C = 0;
        if (h)
            for (int32_t i = 0; i < n; i++)
                E -= (int64_t)h[i] * mk[i];
        for (int64_t e = 0; e < m; e++) {
            int32_t u = eu[e], v = ev[e];
            if (u < 0 || u >= n || v < 0 || v >= n)
                return -1;
            E -= (int64_t)ej[e] * mk[u] * mk[v];
            if (mk[u] != mk[v])
                C += -(int64_t)ej[e];
        }
        energy[k] = E;
        cut[k] = C;
    }
    return 0;
}

int psa_ref_anneal(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   const int32_t *ej, const int32_t *h, int32_t steps,
                   const float *i0, const float *lambda, const float *offset,
                   const uint32_t *thr24, uint64_t seed, int32_t trial_begin,
                   int32_t trial_end, int8_t *spins, int64_t *energy,
                   int64_t *cut)
{
    if (steps < 0)
        return -1;
    int rc = psa_ref_init_spins(n, seed, trial_begin, trial_end, spins);
    if (rc != 0)
        return rc;
    rc = psa_ref_run(n, m, eu, ev, ej, h, i0, lambda, offset, thr24, seed,
                     trial_begin, trial_end, 0, steps, spins);
    if (rc != 0)
        return rc;
    return psa_ref_energy_cut(n, m, eu, ev, ej, h, trial_end - trial_begin,
                              spins, energy, cut);
}
