// kernels.hip -- gfx950 kernels of the pSA hot path.
//
//   init_spins_kernel   initial state: m = +1 iff bit 31 of the INIT word
//   anneal_kernel       persistent sweep kernel: one workgroup owns TPW
//                       trials (1 or 4) of a run and keeps their spins of
//                       every p-bit in LDS, double-buffered; all steps of
//                       the launch run inside the kernel, one workgroup
//                       barrier per step.  The CSR, biases and per-p-bit
//                       factors are staged in LDS as well when they fit.
//   local_field_kernel  L = h + J m (Eq. 3 without I0), for tests
//   energy_cut_kernel   Eq. 2 energy and MAX-CUT value per trial
//   spins_{to,from}_tn  layout conversion [n][t4] <-> [trials][n]
//
// Random words: Philox4x32-10 block of counter (t, i/4, k, purpose) serves
// the four p-bits 4m..4m+3 (m = i/4) of trial k; word i mod 4.  A thread
// therefore always updates a group of four consecutive p-bits ("task" m),
// for one trial (TPW = 1) or for four trials (TPW = 4).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {
namespace {

__device__ __forceinline__ uint32_t load_word(const int8_t *spins, int32_t t4, int32_t i,
                                              int32_t q) {
    return *reinterpret_cast<const uint32_t *>(spins + static_cast<size_t>(i) * t4 + 4 * q);
}

__device__ __forceinline__ void store_word(int8_t *spins, int32_t t4, int32_t i, int32_t q,
                                           uint32_t w) {
    *reinterpret_cast<uint32_t *>(spins + static_cast<size_t>(i) * t4 + 4 * q) = w;
}

__device__ __forceinline__ Words4 block_of(uint32_t t, uint32_t m, uint32_t k, uint32_t tag,
                                           uint32_t k0, uint32_t k1) {
    return philox4x32_10(t, m, k, tag, k0, k1);
}

// ---------------------------------------------------------------------------
// Initial spins: thread per (task m, trial k) over all t4 trials; p-bit
// 4m+p of trial k is +1 iff bit 31 of word p of block (0, m, k, INIT).
// ---------------------------------------------------------------------------
__global__ void init_spins_kernel(int32_t n, int32_t tasks, int32_t t4, uint32_t k0,
                                  uint32_t k1, int8_t *__restrict__ spins) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(tasks) * t4) return;
    const int32_t m = static_cast<int32_t>(idx / t4);
    const int32_t k = static_cast<int32_t>(idx % t4);
    const Words4 w = block_of(0u, static_cast<uint32_t>(m), static_cast<uint32_t>(k), kTagInit,
                              k0, k1);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int32_t i = 4 * m + p;
        if (i < n) spins[static_cast<size_t>(i) * t4 + k] = (ws[p] >> 31) ? int8_t(1) : int8_t(-1);
    }
}

// ---------------------------------------------------------------------------
// Persistent anneal kernel.
// ---------------------------------------------------------------------------
struct AnnealArgs {
    int32_t n, n4, t4, t_begin, t_end;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *val;
    const uint32_t *pk32;
    const uint16_t *pk16;
    const int32_t *h;
    const float *i0;
    const float *lam;
    const float *dlt;
    const uint32_t *thr;
    uint32_t k0, k1;
    int8_t *spins;
};

// Per-p-bit views (LDS or global) used inside the step loop.
template <int CSR>
struct Views {
    const int32_t *row_ptr;
    const int32_t *h;
    const float *lam;
    const float *dlt;
    const uint32_t *thr;
    const int32_t *col;   // kCsrPair
    const int32_t *val;   // kCsrPair
    const uint32_t *pk32; // kCsrPack32
    const uint16_t *pk16; // kCsrPack16
};

// New spin byte of one p-bit for one trial (Eq. 6 with the timing factor as
// an update probability): +1 iff tanh((I0 lambda)(L + delta)) > r.
__device__ __forceinline__ uint32_t decide(float a, float d, int32_t L, uint32_t rword) {
    const float b = static_cast<float>(L) + d;
    const float x = a * b;
    return (tanh_f32(x) > r_of(rword)) ? 0x01u : 0xFFu;
}

// Field of p-bit i for one trial: spins are bytes (TPW = 1).
template <int CSR>
__device__ __forceinline__ int32_t field1(const Views<CSR> &v, int32_t i, const int8_t *cur) {
    int32_t L = v.h[i];
    const int32_t e1 = v.row_ptr[i + 1];
#pragma unroll 4
    for (int32_t e = v.row_ptr[i]; e < e1; ++e) {
        if constexpr (CSR == kCsrPack16) {
            const uint32_t w = v.pk16[e];
            const int32_t s = cur[w >> 1];
            L += (w & 1u) ? -s : s;
        } else if constexpr (CSR == kCsrPack32) {
            const uint32_t w = v.pk32[e];
            L += (static_cast<int32_t>(w) >> 16) * static_cast<int32_t>(cur[w & 0xFFFFu]);
        } else {
            L += v.val[e] * static_cast<int32_t>(cur[v.col[e]]);
        }
    }
    return L;
}

// Fields of p-bit i for four trials: spins are packed words (TPW = 4).
template <int CSR>
__device__ __forceinline__ void field4(const Views<CSR> &v, int32_t i, const uint32_t *cur,
                                       int32_t L[4]) {
    const int32_t hi = v.h[i];
    L[0] = hi;
    L[1] = hi;
    L[2] = hi;
    L[3] = hi;
    const int32_t e1 = v.row_ptr[i + 1];
#pragma unroll 2
    for (int32_t e = v.row_ptr[i]; e < e1; ++e) {
        int32_t J;
        uint32_t wj;
        if constexpr (CSR == kCsrPack16) {
            const uint32_t w = v.pk16[e];
            J = (w & 1u) ? -1 : 1;
            wj = cur[w >> 1];
        } else if constexpr (CSR == kCsrPack32) {
            const uint32_t w = v.pk32[e];
            J = static_cast<int32_t>(w) >> 16;
            wj = cur[w & 0xFFFFu];
        } else {
            J = v.val[e];
            wj = cur[v.col[e]];
        }
        L[0] += J * spin_of(wj, 0);
        L[1] += J * spin_of(wj, 1);
        L[2] += J * spin_of(wj, 2);
        L[3] += J * spin_of(wj, 3);
    }
}

// Task m for one trial k (TPW = 1), spread over LPT consecutive lanes
// (1, 2 or 4): lane `sub` owns the P = 4 / LPT p-bits 4m + sub*P + j and
// returns their new bytes in the low 8P bits.  With the timing gate on and
// LPT >= 2, even lanes draw the r block and odd lanes the gate block of the
// task, and the pair swaps the words the other needs (DPP), so the two
// Philox blocks run side by side instead of one after the other.
template <int CSR, int LPT>
__device__ __forceinline__ uint32_t task1(const Views<CSR> &v, int32_t n, int32_t m,
                                          uint32_t sub, uint32_t k, uint32_t t, float i0t,
                                          const int8_t *cur, uint32_t k0, uint32_t k1) {
    constexpr int P = 4 / LPT;
    bool need_gate = false;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int32_t i = 4 * m + p;
        need_gate |= (i < n) && v.thr[i] < kGateOne;
    }
    const int32_t base = 4 * m + static_cast<int32_t>(sub) * P;
    uint32_t rw[P], gw[P];
    if constexpr (LPT == 1) {
        const Words4 r = block_of(t, static_cast<uint32_t>(m), k, kTagR, k0, k1);
        rw[0] = r.x;
        rw[1] = r.y;
        rw[2] = r.z;
        rw[3] = r.w;
        if (need_gate) {
            const Words4 g = block_of(t, static_cast<uint32_t>(m), k, kTagGate, k0, k1);
            gw[0] = g.x;
            gw[1] = g.y;
            gw[2] = g.z;
            gw[3] = g.w;
        } else {
            gw[0] = gw[1] = gw[2] = gw[3] = 0u;
        }
    } else {
        const uint32_t tag = (need_gate && (sub & 1u)) ? kTagGate : kTagR;
        const Words4 b = block_of(t, static_cast<uint32_t>(m), k, tag, k0, k1);
        if constexpr (LPT == 2) {
            if (need_gate) {  // lane 0 holds r words, lane 1 gate words
                const uint32_t x0 = swap_pair(sub ? b.x : b.z);
                const uint32_t x1 = swap_pair(sub ? b.y : b.w);
                rw[0] = sub ? x0 : b.x;
                rw[1] = sub ? x1 : b.y;
                gw[0] = sub ? b.z : x0;
                gw[1] = sub ? b.w : x1;
            } else {
                rw[0] = sub ? b.z : b.x;
                rw[1] = sub ? b.w : b.y;
                gw[0] = gw[1] = 0u;
            }
        } else {  // LPT == 4: even lanes r block, odd lanes gate block
            const uint32_t own = word_of(b, sub);
            if (need_gate) {
                const uint32_t x = swap_pair(word_of(b, sub ^ 1u));
                const bool even = (sub & 1u) == 0u;
                rw[0] = even ? own : x;
                gw[0] = even ? x : own;
            } else {
                rw[0] = own;
                gw[0] = 0u;
            }
        }
    }
    uint32_t out = 0u;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int32_t i = base + j;
        uint32_t byte = 0x01u;
        if (i < n) {
            byte = static_cast<uint8_t>(cur[i]);
            const uint32_t th = v.thr[i];
            if (th >= kGateOne || fires(gw[j], th)) {
                const int32_t L = field1<CSR>(v, i, cur);
                byte = decide(i0t * v.lam[i], v.dlt[i], L, rw[j]);
            }
        }
        out |= byte << (8 * j);
    }
    return out;
}

// Task m for trials 4q..4q+3 (TPW = 4): writes the four packed words of
// p-bits 4m..4m+3 into nxt.
template <int CSR>
__device__ __forceinline__ void task4(const Views<CSR> &v, int32_t n, int32_t m, int32_t q,
                                      uint32_t t, float i0t, const uint32_t *cur,
                                      uint32_t *nxt, uint32_t k0, uint32_t k1) {
    int32_t L[4][4];
    uint32_t word[4];
    uint32_t th[4];
    float a[4], d[4];
    bool need_gate = false;
    uint32_t valid = 0u;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int32_t i = 4 * m + p;
        const bool ok = i < n;
        valid |= ok ? (1u << p) : 0u;
        word[p] = cur[4 * m + p];
        th[p] = ok ? v.thr[i] : 0u;
        need_gate |= ok && th[p] < kGateOne;
        if (ok) {
            field4<CSR>(v, i, cur, L[p]);
            a[p] = i0t * v.lam[i];
            d[p] = v.dlt[i];
        } else {
            L[p][0] = L[p][1] = L[p][2] = L[p][3] = 0;
            a[p] = 0.0f;
            d[p] = 0.0f;
        }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const uint32_t k = static_cast<uint32_t>(4 * q + kk);
        uint32_t fire = valid;
        if (need_gate) {
            const Words4 g = block_of(t, static_cast<uint32_t>(m), k, kTagGate, k0, k1);
            const uint32_t gw[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
            for (int p = 0; p < 4; ++p)
                if (th[p] < kGateOne && !fires(gw[p], th[p])) fire &= ~(1u << p);
        }
        const Words4 r = block_of(t, static_cast<uint32_t>(m), k, kTagR, k0, k1);
        const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if ((fire >> p) & 1u) {
                const uint32_t byte = decide(a[p], d[p], L[p][kk], rw[p]);
                word[p] = (word[p] & ~(0xFFu << (8 * kk))) | (byte << (8 * kk));
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) nxt[4 * m + p] = word[p];
}

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS carve-up, shared by host planning and the kernel:
//   [spins buffer 0][spins buffer 1]            2 * n4 * TPW bytes
//   [row_ptr n4+4][h n4][lam n4][dlt n4][thr n4] 4-byte entries  (csr_lds)
//   [csr entries nnz * entry bytes]                               (csr_lds)
__host__ __device__ constexpr size_t spins_bytes(int32_t n4, int32_t tpw) {
    return align16(static_cast<size_t>(n4) * tpw);
}
__host__ __device__ constexpr size_t params_bytes(int32_t n4) {
    return static_cast<size_t>(n4 + 4 + 4 * n4) * 4;
}
__host__ __device__ constexpr size_t csr_entry_bytes(int32_t csr) {
    return csr == kCsrPack16 ? 2 : (csr == kCsrPack32 ? 4 : 8);
}

template <int TPW, int LPT, int CSR, bool CSR_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void anneal_kernel(AnnealArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t n = a.n, n4 = a.n4, tasks = n4 / 4;
    const int32_t q = blockIdx.x;  // trial group: trials TPW*q .. TPW*q+TPW-1
    unsigned char *buf0 = smem;
    unsigned char *buf1 = smem + spins_bytes(n4, TPW);

    Views<CSR> v;
    if constexpr (CSR_LDS) {
        int32_t *l_rp = reinterpret_cast<int32_t *>(smem + 2 * spins_bytes(n4, TPW));
        int32_t *l_h = l_rp + n4 + 4;
        float *l_lam = reinterpret_cast<float *>(l_h + n4);
        float *l_dlt = l_lam + n4;
        uint32_t *l_thr = reinterpret_cast<uint32_t *>(l_dlt + n4);
        unsigned char *l_csr = reinterpret_cast<unsigned char *>(l_thr + n4);
        for (int32_t i = threadIdx.x; i <= n; i += BLOCK) l_rp[i] = a.row_ptr[i];
        for (int32_t i = threadIdx.x; i < n; i += BLOCK) {
            l_h[i] = a.h[i];
            l_lam[i] = a.lam[i];
            l_dlt[i] = a.dlt[i];
            l_thr[i] = a.thr[i];
        }
        if constexpr (CSR == kCsrPack16) {
            uint16_t *c = reinterpret_cast<uint16_t *>(l_csr);
            for (int32_t e = threadIdx.x; e < a.nnz; e += BLOCK) c[e] = a.pk16[e];
            v.pk16 = c;
        } else if constexpr (CSR == kCsrPack32) {
            uint32_t *c = reinterpret_cast<uint32_t *>(l_csr);
            for (int32_t e = threadIdx.x; e < a.nnz; e += BLOCK) c[e] = a.pk32[e];
            v.pk32 = c;
        } else {
            int32_t *c = reinterpret_cast<int32_t *>(l_csr);
            int32_t *w = c + a.nnz;
            for (int32_t e = threadIdx.x; e < a.nnz; e += BLOCK) {
                c[e] = a.col[e];
                w[e] = a.val[e];
            }
            v.col = c;
            v.val = w;
        }
        v.row_ptr = l_rp;
        v.h = l_h;
        v.lam = l_lam;
        v.dlt = l_dlt;
        v.thr = l_thr;
    } else {
        v.row_ptr = a.row_ptr;
        v.h = a.h;
        v.lam = a.lam;
        v.dlt = a.dlt;
        v.thr = a.thr;
        v.col = a.col;
        v.val = a.val;
        v.pk32 = a.pk32;
        v.pk16 = a.pk16;
    }

    // spins of this workgroup's trials -> LDS (padding p-bits n..n4-1 = +1)
    if constexpr (TPW == 1) {
        int8_t *s0 = reinterpret_cast<int8_t *>(buf0);
        for (int32_t i = threadIdx.x; i < n4; i += BLOCK)
            s0[i] = i < n ? a.spins[static_cast<size_t>(i) * a.t4 + q] : int8_t(1);
    } else {
        uint32_t *s0 = reinterpret_cast<uint32_t *>(buf0);
        for (int32_t i = threadIdx.x; i < n4; i += BLOCK)
            s0[i] = i < n ? load_word(a.spins, a.t4, i, q) : 0x01010101u;
    }
    __syncthreads();

    unsigned char *cur = buf0;
    unsigned char *nxt = buf1;
    for (int32_t t = a.t_begin; t < a.t_end; ++t) {
        const float i0t = a.i0[t];
        if constexpr (TPW == 1) {
            // all LPT lanes of a task share m, so they enter and leave together
            const uint32_t sub = threadIdx.x % LPT;
            for (int32_t m = threadIdx.x / LPT; m < tasks; m += BLOCK / LPT) {
                const uint32_t b = task1<CSR, LPT>(v, n, m, sub, static_cast<uint32_t>(q),
                                                   static_cast<uint32_t>(t), i0t,
                                                   reinterpret_cast<const int8_t *>(cur), a.k0,
                                                   a.k1);
                if constexpr (LPT == 1) {
                    reinterpret_cast<uint32_t *>(nxt)[m] = b;
                } else if constexpr (LPT == 2) {
                    reinterpret_cast<uint16_t *>(nxt)[2 * m + sub] = static_cast<uint16_t>(b);
                } else {
                    nxt[4 * m + sub] = static_cast<unsigned char>(b);
                }
            }
        } else {
            for (int32_t m = threadIdx.x; m < tasks; m += BLOCK)
                task4<CSR>(v, n, m, q, static_cast<uint32_t>(t), i0t,
                           reinterpret_cast<const uint32_t *>(cur),
                           reinterpret_cast<uint32_t *>(nxt), a.k0, a.k1);
        }
        __syncthreads();
        unsigned char *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }

    if constexpr (TPW == 1) {
        const int8_t *s = reinterpret_cast<const int8_t *>(cur);
        for (int32_t i = threadIdx.x; i < n; i += BLOCK)
            a.spins[static_cast<size_t>(i) * a.t4 + q] = s[i];
    } else {
        const uint32_t *s = reinterpret_cast<const uint32_t *>(cur);
        for (int32_t i = threadIdx.x; i < n; i += BLOCK) store_word(a.spins, a.t4, i, q, s[i]);
    }
}

// ---------------------------------------------------------------------------
// Local field, thread per (i, q); out is [trials][n].
// ---------------------------------------------------------------------------
__global__ void local_field_kernel(int32_t n, int32_t quads, int32_t t4, int32_t trials,
                                   const int32_t *__restrict__ row_ptr,
                                   const int32_t *__restrict__ col,
                                   const int32_t *__restrict__ val,
                                   const int32_t *__restrict__ h,
                                   const int8_t *__restrict__ spins, int32_t *__restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * quads) return;
    const int32_t i = static_cast<int32_t>(idx % n);
    const int32_t q = static_cast<int32_t>(idx / n);
    int32_t L[4] = {h[i], h[i], h[i], h[i]};
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const uint32_t wj = load_word(spins, t4, col[e], q);
#pragma unroll
        for (int k = 0; k < 4; ++k) L[k] += val[e] * spin_of(wj, k);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t trial = 4 * q + k;
        if (trial < trials) out[static_cast<size_t>(trial) * n + i] = L[k];
    }
}

// ---------------------------------------------------------------------------
// Energy and cut, one workgroup per quad of trials.  With
// S_k = sum_i m_i sum_j J_ij m_j (= 2 sum_{i<j} J_ij m_i m_j) and
// W2 = sum_i sum_j J_ij:
//   E_k   = -sum_i h_i m_i - S_k / 2
//   cut_k = sum_{i<j} w_ij [m_i != m_j] = (S_k - W2) / 4     (w = -J)
// ---------------------------------------------------------------------------
constexpr int kEnergyBlock = 256;

__global__ __launch_bounds__(kEnergyBlock) void energy_cut_kernel(
    int32_t n, int32_t t4, int32_t trials, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const int32_t *__restrict__ val,
    const int32_t *__restrict__ h, int64_t w2, const int8_t *__restrict__ spins,
    int64_t *__restrict__ energy, int64_t *__restrict__ cut) {
    const int32_t q = blockIdx.x;
    int64_t s[4] = {0, 0, 0, 0};
    int64_t hm[4] = {0, 0, 0, 0};
    for (int32_t i = threadIdx.x; i < n; i += kEnergyBlock) {
        const uint32_t wi = load_word(spins, t4, i, q);
        int32_t L[4] = {0, 0, 0, 0};
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const uint32_t wj = load_word(spins, t4, col[e], q);
#pragma unroll
            for (int k = 0; k < 4; ++k) L[k] += val[e] * spin_of(wj, k);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t mi = spin_of(wi, k);
            s[k] += static_cast<int64_t>(mi * L[k]);
            hm[k] += static_cast<int64_t>(mi * h[i]);
        }
    }
    __shared__ int64_t red[kEnergyBlock / 64][8];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            s[k] += __shfl_down(s[k], off, 64);
            hm[k] += __shfl_down(hm[k], off, 64);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            red[wave][k] = s[k];
            red[wave][4 + k] = hm[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        int64_t S = 0, H = 0;
        for (int w = 0; w < kEnergyBlock / 64; ++w) {
            S += red[w][k];
            H += red[w][4 + k];
        }
        const int32_t trial = 4 * q + k;
        if (trial < trials) {
            energy[trial] = -H - S / 2;
            cut[trial] = (S - w2) / 4;
        }
    }
}

// [n][t4] -> [trials][n]
__global__ void spins_to_tn_kernel(int32_t n, int32_t t4, int32_t trials,
                                   const int8_t *__restrict__ spins, int8_t *__restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * trials) return;
    const int32_t k = static_cast<int32_t>(idx / n);
    const int32_t i = static_cast<int32_t>(idx % n);
    out[idx] = spins[static_cast<size_t>(i) * t4 + k];
}

// [trials][n] -> [n][t4]; padding trials (k >= trials) are left unchanged.
__global__ void spins_from_tn_kernel(int32_t n, int32_t t4, int32_t trials,
                                     const int8_t *__restrict__ in, int8_t *__restrict__ spins) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * trials) return;
    const int32_t k = static_cast<int32_t>(idx / n);
    const int32_t i = static_cast<int32_t>(idx % n);
    spins[static_cast<size_t>(i) * t4 + k] = in[idx];
}

inline unsigned grid_for(int64_t items, int block) {
    return static_cast<unsigned>((items + block - 1) / block);
}

template <int TPW, int LPT, int CSR, bool LDS, int BLOCK>
hipError_t launch_variant(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    auto kern = anneal_kernel<TPW, LPT, CSR, LDS, BLOCK>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(plan.lds_bytes));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(plan.grid), dim3(BLOCK), plan.lds_bytes, stream, args);
    return hipGetLastError();
}

template <int TPW, int LPT, int CSR, bool LDS>
hipError_t launch_block(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    switch (plan.block) {
        case 256: return launch_variant<TPW, LPT, CSR, LDS, 256>(stream, args, plan);
        case 512: return launch_variant<TPW, LPT, CSR, LDS, 512>(stream, args, plan);
        case 1024: return launch_variant<TPW, LPT, CSR, LDS, 1024>(stream, args, plan);
        default: return hipErrorInvalidValue;
    }
}

template <int TPW, int LPT, int CSR>
hipError_t launch_lds(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    return plan.csr_lds ? launch_block<TPW, LPT, CSR, true>(stream, args, plan)
                        : launch_block<TPW, LPT, CSR, false>(stream, args, plan);
}

template <int TPW, int LPT>
hipError_t launch_csr(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    switch (plan.csr) {
        case kCsrPair: return launch_lds<TPW, LPT, kCsrPair>(stream, args, plan);
        case kCsrPack32: return launch_lds<TPW, LPT, kCsrPack32>(stream, args, plan);
        case kCsrPack16: return launch_lds<TPW, LPT, kCsrPack16>(stream, args, plan);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool plan_anneal(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                 int32_t block_req, size_t max_lds, int32_t num_cu, AnnealPlan *plan,
                 std::string *why) {
    AnnealPlan p;
    const int32_t n4 = (g.n + 3) / 4 * 4;
    if (tpw_req == 1 || tpw_req == 4) {
        p.tpw = tpw_req;
    } else {
        // four trials per workgroup amortise the CSR walk over four trials;
        // one trial per workgroup exposes four times the workgroups.
        p.tpw = (run.t4 / 4 >= num_cu) ? 4 : 1;
    }
    p.grid = p.tpw == 4 ? run.t4 / 4 : run.trials;
    const size_t sp = 2 * spins_bytes(n4, p.tpw);
    if (sp > max_lds) {
        if (why)
            *why = "n = " + std::to_string(g.n) + " does not fit the LDS-resident spin state (" +
                   std::to_string(sp) + " > " + std::to_string(max_lds) + " bytes)";
        return false;
    }
    const int32_t kinds[3] = {kCsrPack16, kCsrPack32, kCsrPair};
    int32_t best = kCsrPair;
    for (int32_t c : kinds) {
        if ((c == kCsrPack16 && !g.pk16) || (c == kCsrPack32 && !g.pk32)) continue;
        best = c;
        break;
    }
    p.csr = best;
    p.csr_lds = 0;
    p.lds_bytes = sp;
    const size_t full = sp + params_bytes(n4) + align16(static_cast<size_t>(g.nnz) * csr_entry_bytes(best));
    if (full <= max_lds) {
        p.csr_lds = 1;
        p.lds_bytes = full;
    }
    const int32_t tasks = n4 / 4;
    if (p.tpw == 4) {
        p.lpt = 1;
    } else if (lpt_req == 1 || lpt_req == 2 || lpt_req == 4) {
        p.lpt = lpt_req;
    } else {
        // more lanes per task while the workgroup has lanes to spare: the
        // small-trial runs are latency-bound, not issue-bound
        p.lpt = tasks * 4 <= 1024 ? 4 : (tasks * 2 <= 2048 ? 2 : 1);
    }
    const int32_t lanes = tasks * p.lpt;
    if (block_req == 256 || block_req == 512 || block_req == 1024) {
        p.block = block_req;
    } else {
        p.block = lanes > 512 ? 1024 : (lanes > 256 ? 512 : 256);
    }
    *plan = p;
    return true;
}

hipError_t launch_init_spins(hipStream_t stream, int32_t n, const DevRun &run) {
    const int32_t tasks = (n + 3) / 4;
    const int block = 256;
    hipLaunchKernelGGL(init_spins_kernel, dim3(grid_for(static_cast<int64_t>(tasks) * run.t4, block)),
                       dim3(block), 0, stream, n, tasks, run.t4, run.key0, run.key1, run.spins);
    return hipGetLastError();
}

hipError_t launch_anneal(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const AnnealPlan &plan, int32_t t_begin, int32_t t_end) {
    if (t_end <= t_begin) return hipSuccess;
    AnnealArgs a;
    a.n = g.n;
    a.n4 = (g.n + 3) / 4 * 4;
    a.t4 = run.t4;
    a.t_begin = t_begin;
    a.t_end = t_end;
    a.nnz = static_cast<int32_t>(g.nnz);
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.val = g.val;
    a.pk32 = g.pk32;
    a.pk16 = g.pk16;
    a.h = g.h;
    a.i0 = run.i0;
    a.lam = run.lambda;
    a.dlt = run.delta;
    a.thr = run.thr24;
    a.k0 = run.key0;
    a.k1 = run.key1;
    a.spins = run.spins;
    if (plan.tpw == 4) return launch_csr<4, 1>(stream, a, plan);
    switch (plan.lpt) {
        case 1: return launch_csr<1, 1>(stream, a, plan);
        case 2: return launch_csr<1, 2>(stream, a, plan);
        case 4: return launch_csr<1, 4>(stream, a, plan);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_local_field(hipStream_t stream, const DevGraph &g, const DevRun &run,
                              int32_t *out_tn) {
    const int32_t quads = run.t4 / 4;
    const int block = 256;
    hipLaunchKernelGGL(local_field_kernel, dim3(grid_for(static_cast<int64_t>(g.n) * quads, block)),
                       dim3(block), 0, stream, g.n, quads, run.t4, run.trials, g.row_ptr, g.col,
                       g.val, g.h, run.spins, out_tn);
    return hipGetLastError();
}

hipError_t launch_energy_cut(hipStream_t stream, const DevGraph &g, const DevRun &run,
                             int64_t *energy, int64_t *cut) {
    hipLaunchKernelGGL(energy_cut_kernel, dim3(run.t4 / 4), dim3(kEnergyBlock), 0, stream, g.n,
                       run.t4, run.trials, g.row_ptr, g.col, g.val, g.h, g.w2, run.spins, energy,
                       cut);
    return hipGetLastError();
}

hipError_t launch_spins_to_tn(hipStream_t stream, int32_t n, const DevRun &run, int8_t *out_tn) {
    const int block = 256;
    hipLaunchKernelGGL(spins_to_tn_kernel,
                       dim3(grid_for(static_cast<int64_t>(n) * run.trials, block)), dim3(block), 0,
                       stream, n, run.t4, run.trials, run.spins, out_tn);
    return hipGetLastError();
}

hipError_t launch_spins_from_tn(hipStream_t stream, int32_t n, const DevRun &run,
                                const int8_t *in_tn) {
    const int block = 256;
    hipLaunchKernelGGL(spins_from_tn_kernel,
                       dim3(grid_for(static_cast<int64_t>(n) * run.trials, block)), dim3(block), 0,
                       stream, n, run.t4, run.trials, in_tn, run.spins);
    return hipGetLastError();
}

}  // namespace psa
