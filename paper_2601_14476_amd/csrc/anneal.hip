// anneal.hip -- the persistent pSA sweep kernel (gfx950).
//
// One workgroup owns TPW trials (1 or 4) of a run, keeps their spins of all
// p-bits in LDS (two buffers, one workgroup barrier per step) and runs every
// step of the launch inside the kernel.  Work is split into *tasks*: a task
// is a group of four consecutive p-bits 4m..4m+3, because one Philox block of
// counter (t, m, k, purpose) supplies the words of exactly those four p-bits
// of trial k (word i mod 4).
//
// Edge encodings (CSR):
//   kCsrUnit   (TPW 1, every |J| = 1): spins in LDS as 0/1 bytes u = (m+1)/2
//              with a complemented copy 1-u behind them; edge e of row i is an
//              index ux16[e] = j (J = +1) or n4 + j (J = -1) into that pair of
//              arrays, so sum_j J_ij m_j = 2 sum_e x_e - deg_i with x_e the
//              byte the index selects: one LDS byte load and one add per edge.
//   kCsrPack16 (TPW 4, every |J| = 1, degree <= 255): four trials' 0/1 bytes
//              per word; pk16[e] = j << 1 | (J < 0); x_e = word_j XOR
//              (J < 0 ? 0x01010101 : 0), summed four trials per 32-bit add.
//              With the rows in device memory the sweep reads the per-task
//              ELL groups instead (entry j of a task's four rows in 16 bytes).
//   kCsrPack32 pk32[e] = j | J << 16; spins as +-1 bytes; general weights.
//   kCsrPair   separate col / val arrays; spins as +-1 bytes; general weights.
// Per-p-bit arrays are padded to n4 = 4 ceil(n/4) entries (padding p-bits have
// no edges and never fire), row_ptr to n4 + 4 entries.
//
// One trial per workgroup with every task on lanes of its own (tasks x LPT <=
// BLOCK) runs "resident": a lane keeps its task's constants, the input-stage
// state and (unit weights, LPT 2 or 4: the fast layout below) the LDS
// addresses of its rows' neighbours in registers for the whole launch.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {
namespace {

// Where the kernel reads the graph and per-p-bit factors from (LDS or global).
struct Views {
    const int32_t *row_ptr;
    const int32_t *h;
    const float *lam;
    const float *dlt;
    const uint32_t *thr;
    const int32_t *order;
    const int32_t *col;
    const int32_t *val;
    const uint32_t *pk32;
    const uint16_t *pk16;
    const uint16_t *ux16;
    const uint32_t *ell;
    const int32_t *eptr;
    const int32_t *pp;
};

__device__ __forceinline__ Words4 block_of(uint32_t t, uint32_t m, uint32_t k, uint32_t tag,
                                           uint32_t k0, uint32_t k1) {
    return philox4x32_10(t, m, k, tag, k0, k1);
}

template <int TPW, int CSR>
struct Enc {
    // 0/1 byte encoding in LDS (else +-1 bytes)
    static constexpr bool kU = (CSR == kCsrUnit) || (TPW == 4 && CSR == kCsrPack16);
    // complemented copy behind the spins (TPW 1, unit weights)
    static constexpr bool kMirror = (CSR == kCsrUnit);
};

// ---------------------------------------------------------------------------
// Fast layout of the one-trial sweep (unit weights, LPT = 2 or 4, at most
// 1,024 lanes of tasks): the two spin buffers lie kFastStride bytes apart and
// each holds four copies of the n4 spins, u, 1 - u, 64 u and 64 (1 - u), then
// a zero byte at 4 n4.  A lane that owns its task for the whole launch keeps
// the LDS addresses of its rows' first fast_slots<P>() edges in registers
// (edges of its second row point into the 64x copies, unused slots at the
// zero byte), so one sum of those bytes holds both rows' counts: the low six
// bits and the rest; a lane with one row caches twice as many.  With the buffer distance a constant, the step loop unrolled
// by two reads either buffer through the load's immediate offset.
// ---------------------------------------------------------------------------
constexpr int32_t kFastStride = 8256;  // >= 4 n4 + 1 for every n4 the layout admits
constexpr int kFastSlots = 32;   // two rows per lane (LPT 2)
constexpr int kFastSlots1 = 64;  // one row per lane (LPT 4)
template <int P>
constexpr int fast_chunk() { return P == 1 ? 8 : 4; }  // slots per wave-uniform skip test
static_assert(kFastSlots < 64, "the first row's count must fit the low six bits");
template <int P>
constexpr int fast_slots() { return P == 1 ? kFastSlots1 : kFastSlots; }

__host__ __device__ constexpr bool fast_layout(int32_t tpw, int32_t lpt, int32_t csr, int32_t n4) {
    return tpw == 1 && csr == kCsrUnit && (lpt == 2 || lpt == 4) && (n4 / 4) * lpt <= 1024;
}

typedef const uint8_t __attribute__((address_space(3))) lds_u8;

// LDS byte address of a pointer into the workgroup's LDS.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_u8 *)(p)));
}

template <uint32_t OFF>
__device__ __forceinline__ uint32_t lds_byte(uint32_t addr) {
    return *((lds_u8 *)(uintptr_t)(addr) + OFF);
}

// ---------------------------------------------------------------------------
// Field sums.
// ---------------------------------------------------------------------------

// One trial, +-1 bytes, general weights: L = h + sum_j J_ij m_j over the
// row's edges e0 .. e1-1.
template <int CSR>
__device__ __forceinline__ int32_t field_pm1(const Views &v, int32_t e0, int32_t e1, int32_t h,
                                             const int8_t *cur) {
    int32_t L = h;
#pragma unroll 2
    for (int32_t e = e0; e < e1; ++e) {
        if constexpr (CSR == kCsrPack32) {
            const uint32_t w = v.pk32[e];
            L += (static_cast<int32_t>(w) >> 16) * static_cast<int32_t>(cur[w & 0xFFFFu]);
        } else {
            L += v.val[e] * static_cast<int32_t>(cur[v.col[e]]);
        }
    }
    return L;
}

// One trial, unit weights, mirrored 0/1 bytes: P = 2 rows (or one) with row
// boundaries rp[0..P] and biases h[0..P-1], walked as one contiguous edge
// range.
template <int P, bool BLK>
__device__ __forceinline__ void field_unit(const Views &v, const int32_t *rp, const int32_t *h,
                                           const uint8_t *cur, int32_t L[P]) {
    const int32_t e0 = rp[0];
    if constexpr (BLK) {
        // rows in global memory: aligned blocks of 8 entries (one 16-byte
        // load), entries outside the rows masked out
        const int32_t split = rp[1];
        const int32_t e2 = P == 2 ? rp[2] : split;
        int32_t acc0 = 0, acc1 = 0;
        for (int32_t eb = e0 & ~7; eb < e2; eb += 8) {
            const u32x4 qv = load_global_x4(v.ux16 + eb);
            const uint32_t wv[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t e = eb + j;
                const int32_t x = cur[(wv[j >> 1] >> (16 * (j & 1))) & 0xFFFFu];
                acc0 += (e >= e0 && e < split) ? x : 0;
                if constexpr (P == 2) acc1 += (e >= split && e < e2) ? x : 0;
            }
        }
        L[0] = h[0] + 2 * acc0 - (split - e0);
        if constexpr (P == 2) L[1] = h[1] + 2 * acc1 - (e2 - split);
        return;
    }
    if constexpr (P == 1) {
        const int32_t e1 = rp[1];
        int32_t acc = 0;
#pragma unroll 4
        for (int32_t e = e0; e < e1; ++e) acc += cur[v.ux16[e]];
        L[0] = h[0] + 2 * acc - (e1 - e0);
    } else {
        const int32_t split = rp[1];
        const int32_t e2 = rp[2];
        int32_t acc = 0, acc0 = 0;
#pragma unroll 4
        for (int32_t e = e0; e < e2; ++e) {
            acc += cur[v.ux16[e]];
            acc0 = (e == split - 1) ? acc : acc0;
        }
        L[0] = h[0] + 2 * acc0 - (split - e0);
        L[1] = h[1] + 2 * (acc - acc0) - (e2 - split);
    }
}

// Unit weights, one trial: the first kCacheEdges edge indices of a lane's
// pair of rows (or one row), two 16-bit indices per register, kept across the
// steps of a launch by a lane that owns its task throughout.  Entries past the
// rows hold index 0 (a valid byte); bit j of sel[r] says entry j belongs to
// row r.
constexpr int kCacheEdges = 16;
struct EdgeCache {
    uint32_t w[kCacheEdges / 2];
    uint32_t sel[2];
};

__device__ __forceinline__ EdgeCache load_edge_cache(const Views &v, int32_t e0, int32_t split,
                                                     int32_t e2) {
    EdgeCache c;
#pragma unroll
    for (int j = 0; j < kCacheEdges / 2; ++j) {
        const int32_t e = e0 + 2 * j;
        const uint32_t lo = e < e2 ? v.ux16[e] : 0u;
        const uint32_t hi = e + 1 < e2 ? v.ux16[e + 1] : 0u;
        c.w[j] = lo | (hi << 16);
    }
    auto below = [](int32_t cnt) -> uint32_t {
        return cnt >= kCacheEdges ? (1u << kCacheEdges) - 1u : (1u << cnt) - 1u;
    };
    c.sel[0] = below(split - e0);
    c.sel[1] = below(e2 - e0) & ~c.sel[0];
    return c;
}

// field_unit with the first kCacheEdges indices from registers: every cached
// byte load is issued at once, the 0/1 bytes are gathered into a bit pattern
// and each row's share counted with one popcount; longer rows finish from the
// edge array.
template <int P, bool BLK>
__device__ __forceinline__ void field_unit_cached(const Views &v, const int32_t *rp, const int32_t *h,
                                                  const EdgeCache &c, const uint8_t *cur,
                                                  int32_t L[P]) {
    const int32_t e0 = rp[0];
    const int32_t split = rp[1];
    const int32_t e2 = P == 2 ? rp[2] : split;
    uint32_t bits = 0u;
#pragma unroll
    for (int j = 0; j < kCacheEdges; ++j)
        bits |= static_cast<uint32_t>(cur[(c.w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu]) << j;
    int32_t acc0 = __builtin_popcount(bits & c.sel[0]);
    int32_t acc1 = P == 2 ? __builtin_popcount(bits & c.sel[1]) : 0;
    for (int32_t e = e0 + kCacheEdges; e < e2; ++e) {
        const uint32_t idx = BLK ? *(const uint16_t __attribute__((address_space(1))) *)(v.ux16 + e)
                                 : v.ux16[e];
        const int32_t x = cur[idx];
        acc0 += e < split ? x : 0;
        if constexpr (P == 2) acc1 += e >= split ? x : 0;
    }
    L[0] = h[0] + 2 * acc0 - (split - e0);
    if constexpr (P == 2) L[1] = h[1] + 2 * acc1 - (e2 - split);
}

// Fast layout: the lane's slot addresses (into buffer 0) for rows rp[0..P],
// P = 1 or 2, and the number of fast_chunk<P>()-slot chunks that some lane of the
// wavefront uses (uniform; tasks are ordered heaviest first, so the lanes of a
// wavefront have rows of similar length).
template <int P>
struct FastCache {
    uint32_t a[fast_slots<P>()];
    uint32_t chunks;
};

template <int P>
__device__ __forceinline__ FastCache<P> load_fast_cache(const Views &v, const int32_t *rp, uint32_t base0,
                                                     int32_t n4) {
    FastCache<P> c;
    const int32_t e0 = rp[0], split = rp[1], e2 = rp[P];
#pragma unroll
    for (int j = 0; j < fast_slots<P>(); ++j) {
        const int32_t e = e0 + j;
        uint32_t x = 4u * static_cast<uint32_t>(n4);  // the zero byte
        if (e < e2) x = v.ux16[e] + (e >= split ? 2u * static_cast<uint32_t>(n4) : 0u);
        c.a[j] = base0 + x;
    }
    return c;
}

// Fields of the lane's P rows from the buffer at LDS offset OFF (cur points
// there): the cached slots in one sum, then the edges past them.
template <int P, uint32_t OFF, bool BLK>
__device__ __forceinline__ void field_fast(const Views &v, const int32_t *rp, const int32_t *h,
                                           const FastCache<P> &c, const uint8_t *cur, int32_t L[P]) {
    uint32_t acc = 0u;
    constexpr int K = fast_slots<P>();
    constexpr int C = fast_chunk<P>();
#pragma unroll
    for (int g = 0; g < K / C; ++g) {
        if (static_cast<uint32_t>(g) < c.chunks) {
#pragma unroll
            for (int j = 0; j < C; ++j) acc += lds_byte<OFF>(c.a[C * g + j]);
        }
    }
    const int32_t e0 = rp[0], split = rp[1], e2 = rp[P];
    // one row: the whole sum; two rows: the low six bits and the rest
    int32_t c0 = static_cast<int32_t>(P == 1 ? acc : (acc & 63u));
    int32_t c1 = static_cast<int32_t>(P == 1 ? 0u : (acc >> 6));
    for (int32_t e = e0 + K; e < e2; ++e) {
        const uint32_t idx = BLK ? *(const uint16_t __attribute__((address_space(1))) *)(v.ux16 + e)
                                 : v.ux16[e];
        const int32_t x = cur[idx];
        c0 += e < split ? x : 0;
        c1 += e < split ? 0 : x;
    }
    L[0] = h[0] + 2 * c0 - (split - e0);
    if constexpr (P == 2) L[1] = h[1] + 2 * c1 - (e2 - split);
}

// Four trials, unit weights, 0/1 bytes packed per word (SWAR); degree <= 255.
template <bool BLK>
__device__ __forceinline__ void field_swar(const Views &v, int32_t i, const uint32_t *cur,
                                           int32_t L[4]) {
    const int32_t e0 = v.row_ptr[i], e1 = v.row_ptr[i + 1];
    uint32_t acc = 0u;
    if constexpr (BLK) {
        // row in global memory: aligned blocks of 8 entries (one 16-byte
        // load), entries outside the row masked out
        for (int32_t eb = e0 & ~7; eb < e1; eb += 8) {
            const u32x4 qv = load_global_x4(v.pk16 + eb);
            const uint32_t wv[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t e = eb + j;
                const uint32_t w = (wv[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                const uint32_t x = cur[w >> 1] ^ ((w & 1u) * 0x01010101u);
                acc += (e >= e0 && e < e1) ? x : 0u;
            }
        }
    } else {
#pragma unroll 2
        for (int32_t e = e0; e < e1; ++e) {
            const uint32_t w = v.pk16[e];
            acc += cur[w >> 1] ^ ((w & 1u) * 0x01010101u);
        }
    }
    const int32_t base = v.h[i] - (e1 - e0);
    L[0] = base + 2 * static_cast<int32_t>(acc & 0xFFu);
    L[1] = base + 2 * static_cast<int32_t>((acc >> 8) & 0xFFu);
    L[2] = base + 2 * static_cast<int32_t>((acc >> 16) & 0xFFu);
    L[3] = base + 2 * static_cast<int32_t>(acc >> 24);
}

// Four trials, unit weights, the task's rows from the per-task ELL array in
// device memory (16 bytes per group: entry j of the four rows, col | (J < 0)
// << 31, the zero word past a row's end): no masks, one 16-byte load per group.
__device__ __forceinline__ void field_ell(const Views &v, int32_t m, const uint32_t *cur,
                                          uint32_t acc[4]) {
    const unsigned char *cb = reinterpret_cast<const unsigned char *>(cur);
    const int32_t g0 = v.eptr[m], g1 = v.eptr[m + 1];
    // groups eight (then four) at a time: their 16-byte loads in flight
    // together, then their neighbour words; a last partial chunk of four
    // reads its missing groups at the task's last group and adds nothing
    // for them
    auto chunk = [&](auto u_tag, int32_t gi, bool tail) __attribute__((always_inline)) {
        constexpr int U = decltype(u_tag)::value;
        u32x4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = load_global_x4(v.ell + 4 * static_cast<size_t>(tail ? min(gi + u, g1 - 1) : gi + u));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ev[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                // word index << 2 drops the sign bit; the sign, spread by an
                // arithmetic shift, complements the four 0/1 bytes
                const uint32_t w = *reinterpret_cast<const uint32_t *>(cb + (ev[p] << 2));
                const uint32_t neg = static_cast<uint32_t>(static_cast<int32_t>(ev[p]) >> 31);
                const uint32_t c = w ^ (neg & 0x01010101u);
                acc[p] += (!tail || gi + u < g1) ? c : 0u;
            }
        }
    };
    int32_t gi = g0;
    for (; gi + 8 <= g1; gi += 8) chunk(std::integral_constant<int, 8>{}, gi, false);
    if (gi + 4 <= g1) {
        chunk(std::integral_constant<int, 4>{}, gi, false);
        gi += 4;
    }
    if (gi < g1) chunk(std::integral_constant<int, 4>{}, gi, true);
}

// Four trials, +-1 bytes packed per word, general weights.
template <int CSR>
__device__ __forceinline__ void field_words(const Views &v, int32_t i, const uint32_t *cur,
                                            int32_t L[4]) {
    const int32_t hi = v.h[i];
    L[0] = L[1] = L[2] = L[3] = hi;
    const int32_t e1 = v.row_ptr[i + 1];
#pragma unroll 2
    for (int32_t e = v.row_ptr[i]; e < e1; ++e) {
        int32_t J;
        uint32_t wj;
        if constexpr (CSR == kCsrPack32) {
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

// ---------------------------------------------------------------------------
// Random words of a task for one trial.  With LPT lanes per task, lane `sub`
// needs the words of its P = 4/LPT p-bits sub*P .. sub*P+P-1.  When the gate
// is on and LPT >= 2, even lanes draw the r block and odd lanes the gate
// block, and each pair swaps the words the other needs (DPP), so the two
// Philox blocks run side by side.
// ---------------------------------------------------------------------------
template <int LPT>
__device__ __forceinline__ void task_words(uint32_t t, uint32_t m, uint32_t k, uint32_t sub,
                                           bool need_gate, uint32_t k0, uint32_t k1,
                                           uint32_t rw[4 / LPT], uint32_t gw[4 / LPT]) {
    if constexpr (LPT == 1) {
        const Words4 r = block_of(t, m, k, kTagR, k0, k1);
        rw[0] = r.x;
        rw[1] = r.y;
        rw[2] = r.z;
        rw[3] = r.w;
        gw[0] = gw[1] = gw[2] = gw[3] = 0u;
        if (need_gate) {
            const Words4 g = block_of(t, m, k, kTagGate, k0, k1);
            gw[0] = g.x;
            gw[1] = g.y;
            gw[2] = g.z;
            gw[3] = g.w;
        }
    } else {
        const uint32_t tag = (need_gate && (sub & 1u)) ? kTagGate : kTagR;
        const Words4 b = block_of(t, m, k, tag, k0, k1);
        if constexpr (LPT == 2) {
            if (need_gate) {  // lane 0 holds the r words, lane 1 the gate words
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
}

__device__ __forceinline__ bool any_gate(const uint32_t *thr, int32_t m) {
    const uint4 th = *reinterpret_cast<const uint4 *>(thr + 4 * m);
    return (th.x < kGateOne) | (th.y < kGateOne) | (th.z < kGateOne) | (th.w < kGateOne);
}

// ---------------------------------------------------------------------------
// One trial per workgroup.  TaskConst holds what lane `sub` of task m reads
// of the graph and factors for its P = 4/LPT p-bits base .. base+P-1: the same
// at every step, so a lane that owns one task for the whole launch loads it
// once and keeps it in registers.
// ---------------------------------------------------------------------------
template <int P>
struct TaskConst {
    int32_t m, base;
    int32_t rp[P + 1];  // row_ptr[base .. base+P]
    int32_t h[P];
    float lam[P], dlt[P];
    uint32_t thr[P];
    bool need_gate;     // some p-bit of the task (all four) has a timing gate
};

template <int LPT>
__device__ __forceinline__ TaskConst<4 / LPT> load_task(const Views &v, int32_t m, uint32_t sub) {
    constexpr int P = 4 / LPT;
    TaskConst<P> c;
    c.m = m;
    c.base = 4 * m + static_cast<int32_t>(sub) * P;
#pragma unroll
    for (int j = 0; j <= P; ++j) c.rp[j] = v.row_ptr[c.base + j];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        c.h[j] = v.h[c.base + j];
        c.lam[j] = v.lam[c.base + j];
        c.dlt[j] = v.dlt[c.base + j];
        c.thr[j] = v.thr[c.base + j];
    }
    c.need_gate = any_gate(v.thr, m);
    return c;
}

// Lane `sub` of task c.m updates its P p-bits at step t and returns their new
// bytes (in the LDS encoding) in the low 8P bits.
// Input-stage state a resident lane keeps in registers for its P p-bits:
// TApSA window sums (the fields of the last min(t+1, alpha) steps, the
// current one included) and SpSA held pre-activations.
template <int P>
struct LaneInput {
    int32_t wsum[P];
    float held[P];
};

// Field sources of the one-trial update.
enum : int { kFieldPlain = 0, kFieldEdgeCache = 1, kFieldFast0 = 2, kFieldFast1 = 3 };

template <int CSR, int LPT, int ALG, bool BLK, int FIELD, bool LRING = false>
__device__ __forceinline__ uint32_t task_one_trial(const Views &v, const TaskConst<4 / LPT> &c,
                                                   const EdgeCache *ec, const FastCache<4 / LPT> *fc,
                                                   LaneInput<4 / LPT> *li, int32_t *lring, uint32_t sub, uint32_t k,
                                                   uint32_t t, float i0t, const unsigned char *cur,
                                                   uint32_t k0, uint32_t k1, const InputState &st) {
    constexpr int P = 4 / LPT;
    constexpr bool kU = Enc<1, CSR>::kU;
    // resident lanes carry the input stage in registers (li)
    constexpr bool RES = FIELD != kFieldPlain;
    const int32_t base = c.base;
    if constexpr (ALG == kAlgPeriod) {
        // t is the sub-step; p-bits whose period does not divide it hold
        bool anyf = false;
#pragma unroll
        for (int j = 0; j < P; ++j) anyf |= period_fires(t, c.thr[j]);
        if (!anyf) {
            uint32_t out = 0u;
#pragma unroll
            for (int j = 0; j < P; ++j) out |= static_cast<uint32_t>(cur[base + j]) << (8 * j);
            return out;
        }
    }
    // TApSA, resident: the field that leaves the window (step t - alpha) sits
    // in the slot this step's field takes; its load is issued first
    int32_t tap_old[P];
    int32_t *tap_w[P];
    if constexpr (ALG == kAlgTapsa && RES) {
        const uint32_t al = static_cast<uint32_t>(st.alpha);
        const uint32_t slot = t % al;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if constexpr (LRING)
                tap_w[j] = lring + static_cast<size_t>(base + j) * al + slot;
            else
                tap_w[j] = st.ring + ((static_cast<size_t>(k >> 2) * st.n4 + base + j) * al + slot) * 4 + (k & 3u);
            tap_old[j] = t >= al ? *tap_w[j] : 0;
        }
    } else {
        (void)lring;
    }
    const bool need_gate = ALG != kAlgPeriod && c.need_gate;
    uint32_t rw[P], gw[P], sw[P];
    task_words<LPT>(t, static_cast<uint32_t>(c.m), k, sub, need_gate, k0, k1, rw, gw);
#pragma unroll
    for (int j = 0; j < P; ++j) sw[j] = 0u;
    if (ALG == kAlgSpsa && t > 0) {
        const Words4 b = block_of(t, static_cast<uint32_t>(c.m), k, kTagStall, k0, k1);
#pragma unroll
        for (int j = 0; j < P; ++j) sw[j] = word_of(b, sub * P + j);
    }
    int32_t L[P];
    if constexpr (CSR == kCsrUnit && (FIELD == kFieldFast0 || FIELD == kFieldFast1) && P <= 2) {
        (void)ec;
        field_fast<P, FIELD == kFieldFast0 ? 0u : static_cast<uint32_t>(kFastStride), BLK>(
            v, c.rp, c.h, *fc, cur, L);
    } else if constexpr (CSR == kCsrUnit && FIELD == kFieldEdgeCache) {
        (void)fc;
        if constexpr (P == 4) {
            field_unit_cached<2, BLK>(v, c.rp, c.h, ec[0], cur, L);
            field_unit_cached<2, BLK>(v, c.rp + 2, c.h + 2, ec[1], cur, L + 2);
        } else {
            field_unit_cached<P, BLK>(v, c.rp, c.h, ec[0], cur, L);
        }
    } else if constexpr (CSR == kCsrUnit) {
        (void)ec, (void)fc;
        if constexpr (P == 4) {
            field_unit<2, BLK>(v, c.rp, c.h, cur, L);
            field_unit<2, BLK>(v, c.rp + 2, c.h + 2, cur, L + 2);
        } else {
            field_unit<P, BLK>(v, c.rp, c.h, cur, L);
        }
    } else {
        (void)ec, (void)fc;
#pragma unroll
        for (int j = 0; j < P; ++j)
            L[j] = field_pm1<CSR>(v, c.rp[j], c.rp[j + 1], c.h[j], reinterpret_cast<const int8_t *>(cur));
    }
    // pre-activations, then the P decisions from the tanh estimate; when
    // some lane of the wave holds an estimate within 2^-16 of r, the P are
    // retaken with the exact recipe -- one uniform branch per task, none per
    // p-bit (pbit_up's decisions either way)
    float xv[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int32_t i = base + j;
        float x;
        if constexpr (ALG == kAlgTapsa && RES) {
            // the window sum advanced by the entering and the leaving field
            li->wsum[j] += L[j] - tap_old[j];
            *tap_w[j] = L[j];
            const uint32_t al = static_cast<uint32_t>(st.alpha);
            const uint32_t count = t + 1 < al ? t + 1 : al;
            const float mean = static_cast<float>(li->wsum[j]) / static_cast<float>(count);
            x = (i0t * c.lam[j]) * (mean + c.dlt[j]);
        } else if constexpr (ALG == kAlgSpsa && RES) {
            const float fresh = (i0t * c.lam[j]) * (static_cast<float>(L[j]) + c.dlt[j]);
            x = (t > 0 && (sw[j] >> 8) < st.s24) ? li->held[j] : fresh;
            li->held[j] = x;
        } else {
            (void)li;
            x = input_of<ALG>(i0t * c.lam[j], c.dlt[j], L[j], st, i, k, t, sw[j]);
        }
        xv[j] = x;
    }
    bool up[P];
    bool close = false;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const float diff = tanh_estimate_minus(xv[j], r_of(rw[j]));
        close = close || !estimate_decides(diff);
        up[j] = diff > 0.0f;
    }
    if (__ballot(close) != 0u) {
#pragma unroll
        for (int j = 0; j < P; ++j) up[j] = tanh_f32(xv[j]) > r_of(rw[j]);
    }
    uint32_t out = 0u;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const uint32_t old = cur[base + j];
        const uint32_t th = c.thr[j];
        const bool fire = ALG == kAlgPeriod ? period_fires(t, th) : (th >= kGateOne || fires(gw[j], th));
        const uint32_t nb = kU ? (up[j] ? 1u : 0u) : (up[j] ? 0x01u : 0xFFu);
        out |= (fire ? nb : old) << (8 * j);
    }
    return out;
}

// ---------------------------------------------------------------------------
// Four trials per workgroup: one lane per task updates 4 p-bits x 4 trials and
// writes the four packed words of the next step.
// ---------------------------------------------------------------------------
template <int CSR, int ALG, bool BLK>
__device__ __forceinline__ void task_four_trials(const Views &v, int32_t m, int32_t q, uint32_t t,
                                                 float i0t, const uint32_t *cur, uint32_t *nxt,
                                                 uint32_t k0, uint32_t k1, const InputState &st) {
    constexpr bool kU = Enc<4, CSR>::kU;
    // unit weights with the rows in device memory: the ELL rows and the
    // packed per-p-bit constants (h - deg, lambda, delta, thr24)
    constexpr bool kEll = CSR == kCsrPack16 && BLK;
    int32_t L[4][4];
    uint32_t word[4], th[4];
    float a[4], d[4];
    int32_t hd[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int32_t i = 4 * m + p;
        word[p] = cur[i];
        if constexpr (kEll) {
            const u32x4 c = load_global_x4(v.pp + 4 * static_cast<size_t>(i));
            hd[p] = static_cast<int32_t>(c.x);
            a[p] = i0t * __uint_as_float(c.y);
            d[p] = __uint_as_float(c.z);
            th[p] = c.w;
        } else {
            th[p] = v.thr[i];
        }
    }
    if constexpr (ALG == kAlgPeriod) {
        // t is the sub-step; p-bits whose period does not divide it hold
        if (!(period_fires(t, th[0]) | period_fires(t, th[1]) | period_fires(t, th[2]) |
              period_fires(t, th[3]))) {
#pragma unroll
            for (int p = 0; p < 4; ++p) nxt[4 * m + p] = word[p];
            return;
        }
    }
    uint32_t acc_ell[4] = {0u, 0u, 0u, 0u};
    float hdf[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (kEll) {
        field_ell(v, m, cur, acc_ell);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            hdf[p] = static_cast<float>(hd[p]);
            if constexpr (ALG != kAlgPsa) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    L[p][kk] = hd[p] + 2 * static_cast<int32_t>((acc_ell[p] >> (8 * kk)) & 0xFFu);
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int32_t i = 4 * m + p;
            a[p] = i0t * v.lam[i];
            d[p] = v.dlt[i];
            if constexpr (CSR == kCsrPack16)
                field_swar<BLK>(v, i, cur, L[p]);
            else
                field_words<CSR>(v, i, cur, L[p]);
        }
    }
    const bool need_gate = ALG != kAlgPeriod && ((th[0] < kGateOne) | (th[1] < kGateOne) |
                                                 (th[2] < kGateOne) | (th[3] < kGateOne));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const uint32_t k = static_cast<uint32_t>(4 * q + kk);
        uint32_t gw[4] = {0u, 0u, 0u, 0u};
        if (need_gate) {
            const Words4 g = block_of(t, static_cast<uint32_t>(m), k, kTagGate, k0, k1);
            gw[0] = g.x;
            gw[1] = g.y;
            gw[2] = g.z;
            gw[3] = g.w;
        }
        const Words4 r = block_of(t, static_cast<uint32_t>(m), k, kTagR, k0, k1);
        const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
        uint32_t sw[4] = {0u, 0u, 0u, 0u};
        if (ALG == kAlgSpsa && t > 0) {
            const Words4 b = block_of(t, static_cast<uint32_t>(m), k, kTagStall, k0, k1);
            sw[0] = b.x;
            sw[1] = b.y;
            sw[2] = b.z;
            sw[3] = b.w;
        }
        // the four decisions from the tanh estimate; when some lane of the
        // wave holds an estimate within 2^-16 of r, the four are retaken
        // with the exact recipe -- one uniform branch per block, none per
        // p-bit (pbit_up's decisions either way)
        float x[4];
        bool up[4];
        bool close = false;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if constexpr (kEll && ALG == kAlgPsa) {
                // (float)L from the byte count directly: 2 count + (h - deg) is
                // an integer below 2^24 in magnitude, so the one fma is exact
                // and equals the converted field; then the pre-activation as
                // everywhere, a ((float)L + delta)
                const float cnt = static_cast<float>((acc_ell[p] >> (8 * kk)) & 0xFFu);
                const float Lf = fmaf(2.0f, cnt, hdf[p]);
                x[p] = a[p] * (Lf + d[p]);
            } else {
                x[p] = input_of<ALG>(a[p], d[p], L[p][kk], st, 4 * m + p, k, t, sw[p]);
            }
            const float diff = tanh_estimate_minus(x[p], r_of(rw[p]));
            close = close || !estimate_decides(diff);
            up[p] = diff > 0.0f;
        }
        if (__ballot(close) != 0u) {
#pragma unroll
            for (int p = 0; p < 4; ++p) up[p] = tanh_f32(x[p]) > r_of(rw[p]);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const bool fire = ALG == kAlgPeriod ? period_fires(t, th[p])
                                                : (th[p] >= kGateOne || fires(gw[p], th[p]));
            const uint32_t nb = kU ? (up[p] ? 1u : 0u) : (up[p] ? 0x01u : 0xFFu);
            if (fire) word[p] = (word[p] & ~(0xFFu << (8 * kk))) | (nb << (8 * kk));
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) nxt[4 * m + p] = word[p];
}

// ---------------------------------------------------------------------------
// LDS carve-up (also used by the host planner):
//   [buffer 0][buffer 1]                       2 * spin_stride
//   [TApSA windows]                            ring_lds_bytes
//   [row_ptr n4+4][h n4][lam n4][dlt n4][thr n4][order tasks rounded to 4]  (csr_lds)
//   [edges: nnz * edge_bytes]                                               (csr_lds)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ constexpr size_t spin_buf_bytes(int32_t n4, int32_t tpw, int32_t csr) {
    // four trials per workgroup: one more word, kept zero (ELL padding entries)
    return align16(static_cast<size_t>(n4) * tpw * (csr == kCsrUnit ? 2 : 1) + (tpw == 4 ? 4 : 0));
}

// Distance between the two spin buffers.
__host__ __device__ constexpr size_t spin_stride(int32_t n4, int32_t tpw, int32_t lpt, int32_t csr) {
    return fast_layout(tpw, lpt, csr, n4) ? static_cast<size_t>(kFastStride) : spin_buf_bytes(n4, tpw, csr);
}

// TApSA windows of a fast-layout run in LDS ([n4][alpha] int32 of the
// workgroup's trial, behind the spin buffers) when they take at most 64 KB;
// else they stay in device memory.
__host__ __device__ constexpr size_t ring_lds_bytes(int32_t n4, int32_t tpw, int32_t lpt, int32_t csr,
                                                    bool has_ring, int32_t alpha) {
    return (has_ring && fast_layout(tpw, lpt, csr, n4) &&
            static_cast<size_t>(n4) * static_cast<size_t>(alpha) * 4 <= 65536)
               ? align16(static_cast<size_t>(n4) * static_cast<size_t>(alpha) * 4)
               : 0;
}

__host__ __device__ constexpr size_t params_bytes(int32_t n4) {
    return static_cast<size_t>(n4 + 4 + 4 * n4 + (n4 / 4 + 3) / 4 * 4) * 4;
}

__host__ __device__ constexpr size_t edge_bytes(int32_t csr) {
    return (csr == kCsrPack16 || csr == kCsrUnit) ? 2 : (csr == kCsrPack32 ? 4 : 8);
}

// Whole run of one workgroup: trial group q of the run described by `a`,
// steps a.t_begin .. a.t_end-1.  `smem` is the dynamic LDS of the launch.
template <int TPW, int LPT, int CSR, bool CSR_LDS, int BLOCK>
__device__ __forceinline__ void anneal_body(const AnnealArgs &a, int32_t q, unsigned char *smem) {
    using E = Enc<TPW, CSR>;
    const int32_t n = a.n, n4 = a.n4, tasks = a.tasks;
    constexpr bool kFastKind = TPW == 1 && CSR == kCsrUnit && (LPT == 2 || LPT == 4);
    const bool fast_lay = kFastKind && fast_layout(TPW, LPT, CSR, n4);
    const size_t sb = spin_stride(n4, TPW, LPT, CSR);
    const size_t ring_res = ring_lds_bytes(n4, TPW, LPT, CSR, a.ring != nullptr, a.alpha);
    unsigned char *buf0 = smem;
    unsigned char *buf1 = smem + sb;
    int32_t *lring = reinterpret_cast<int32_t *>(smem + 2 * sb);

    Views v;
    if constexpr (CSR_LDS) {
        int32_t *l_rp = reinterpret_cast<int32_t *>(smem + 2 * sb + ring_res);
        int32_t *l_h = l_rp + n4 + 4;
        float *l_lam = reinterpret_cast<float *>(l_h + n4);
        float *l_dlt = l_lam + n4;
        uint32_t *l_thr = reinterpret_cast<uint32_t *>(l_dlt + n4);
        int32_t *l_ord = reinterpret_cast<int32_t *>(l_thr + n4);
        unsigned char *l_edges = reinterpret_cast<unsigned char *>(l_ord + (tasks + 3) / 4 * 4);
        for (int32_t i = threadIdx.x; i < n4 + 4; i += BLOCK) l_rp[i] = a.row_ptr[i];
        for (int32_t i = threadIdx.x; i < n4; i += BLOCK) {
            l_h[i] = a.h[i];
            l_lam[i] = a.lam[i];
            l_dlt[i] = a.dlt[i];
            l_thr[i] = a.thr[i];
        }
        for (int32_t i = threadIdx.x; i < tasks; i += BLOCK) l_ord[i] = a.order[i];
        if constexpr (CSR == kCsrUnit || CSR == kCsrPack16) {
            const uint16_t *src = CSR == kCsrUnit ? a.ux16 : a.pk16;
            uint16_t *c = reinterpret_cast<uint16_t *>(l_edges);
            for (int32_t e = threadIdx.x; e < a.nnz; e += BLOCK) c[e] = src[e];
            v.ux16 = c;
            v.pk16 = c;
        } else if constexpr (CSR == kCsrPack32) {
            uint32_t *c = reinterpret_cast<uint32_t *>(l_edges);
            for (int32_t e = threadIdx.x; e < a.nnz; e += BLOCK) c[e] = a.pk32[e];
            v.pk32 = c;
        } else {
            int32_t *c = reinterpret_cast<int32_t *>(l_edges);
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
        v.order = l_ord;
    } else {
        v.row_ptr = a.row_ptr;
        v.h = a.h;
        v.lam = a.lam;
        v.dlt = a.dlt;
        v.thr = a.thr;
        v.order = a.order;
        v.col = a.col;
        v.val = a.val;
        v.pk32 = a.pk32;
        v.pk16 = a.pk16;
        v.ux16 = a.ux16;
    }
    v.ell = a.ell;
    v.eptr = a.eptr;
    v.pp = a.pp;

    // spins of this workgroup's trials -> LDS (padding p-bits = +1)
    if constexpr (TPW == 1) {
        for (int32_t i = threadIdx.x; i < n4; i += BLOCK) {
            const int8_t s = i < n ? a.spins[static_cast<size_t>(i) * a.t4 + q] : int8_t(1);
            if constexpr (E::kU) {
                const unsigned char u = s > 0 ? 1 : 0;
                buf0[i] = u;
                if constexpr (E::kMirror) buf0[n4 + i] = u ^ 1u;
                if (fast_lay) {
                    buf0[2 * n4 + i] = static_cast<unsigned char>(u << 6);
                    buf0[3 * n4 + i] = static_cast<unsigned char>((u ^ 1u) << 6);
                }
            } else {
                buf0[i] = static_cast<unsigned char>(s);
            }
        }
        if (fast_lay && threadIdx.x == 0) {
            buf0[4 * n4] = 0;
            buf1[4 * n4] = 0;
        }
    } else {
        uint32_t *s0 = reinterpret_cast<uint32_t *>(buf0);
        for (int32_t i = threadIdx.x; i < n4; i += BLOCK) {
            const uint32_t w = i < n ? *reinterpret_cast<const uint32_t *>(
                                           a.spins + static_cast<size_t>(i) * a.t4 + 4 * q)
                                     : 0x01010101u;
            s0[i] = E::kU ? ((~w >> 7) & 0x01010101u) : w;
        }
        if (threadIdx.x == 0) {
            s0[n4] = 0u;
            reinterpret_cast<uint32_t *>(buf1)[n4] = 0u;
        }
    }
    __syncthreads();

    unsigned char *cur = buf0;
    unsigned char *nxt = buf1;
    const InputState st{a.xs, a.stall24, a.ring, a.alpha, n4};

    // One trial per workgroup: update the P p-bits of one task and store them
    // (and the complemented copy) into the next buffer.
    constexpr int P = 4 / LPT;
    const uint32_t sub = threadIdx.x % LPT;
    auto one_trial_step = [&](auto alg_tag, auto cached_tag, const TaskConst<P> &c,
                              const EdgeCache *ec, LaneInput<P> *li, uint32_t tau, float i0t,
                              uint32_t k0, uint32_t k1, const unsigned char *from, unsigned char *to)
                              __attribute__((always_inline)) {
        constexpr int ALG = decltype(alg_tag)::value;
        constexpr bool CACHED = decltype(cached_tag)::value;
        const uint32_t b = task_one_trial<CSR, LPT, ALG, !CSR_LDS, CACHED ? kFieldEdgeCache : kFieldPlain>(
            v, c, ec, nullptr, li, nullptr, sub, static_cast<uint32_t>(q), tau, i0t, from, k0, k1, st);
        const int32_t at = c.base;
        if constexpr (P == 4) {
            *reinterpret_cast<uint32_t *>(to + at) = b;
            if constexpr (E::kMirror) *reinterpret_cast<uint32_t *>(to + n4 + at) = b ^ 0x01010101u;
        } else if constexpr (P == 2) {
            *reinterpret_cast<uint16_t *>(to + at) = static_cast<uint16_t>(b);
            if constexpr (E::kMirror)
                *reinterpret_cast<uint16_t *>(to + n4 + at) = static_cast<uint16_t>(b ^ 0x0101u);
        } else {
            to[at] = static_cast<unsigned char>(b);
            if constexpr (E::kMirror) to[n4 + at] = static_cast<unsigned char>(b ^ 1u);
        }
    };
    // When every task has a slot of its own (tasks x LPT <= BLOCK), a lane
    // keeps its task's constants in registers for the whole launch.
    const bool resident = TPW == 1 && tasks * LPT <= BLOCK;
    const bool owns = resident && static_cast<int32_t>(threadIdx.x) / LPT < tasks;
    // resident lanes in the fast layout (LPT 2 or 4) sum cached slots; other
    // resident lanes (LPT 1) walk cached edge indices
    const bool fast = fast_lay && resident;
    TaskConst<P> own{};
    EdgeCache own_edges[P == 4 ? 2 : 1] = {};
    FastCache<P> own_fast = {};
    LaneInput<P> own_in = {};
    if (owns) {
        own = load_task<LPT>(v, v.order[threadIdx.x / LPT], sub);
        // input-stage state of the lane's p-bits: the TApSA window sums up to
        // step t_begin - 1 from the ring, the SpSA held inputs
        const size_t row0 = static_cast<size_t>(q >> 2) * n4 + own.base;
        if (a.ring != nullptr) {
            const int32_t al = a.alpha;
            const int32_t cnt = a.t_begin < al ? a.t_begin : al;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                int32_t sum = 0;
                for (int32_t i = 0; i < cnt; ++i)
                    sum += a.ring[((row0 + j) * al + (a.t_begin - 1 - i) % al) * 4 + (q & 3)];
                own_in.wsum[j] = sum;
            }
        }
        if (a.xs != nullptr) {
#pragma unroll
            for (int j = 0; j < P; ++j) own_in.held[j] = a.xs[(row0 + j) * 4 + (q & 3)];
        }
        if constexpr (kFastKind) {
            if (fast) own_fast = load_fast_cache<P>(v, own.rp, lds_addr(smem), n4);
        }
        if constexpr (CSR == kCsrUnit) {
            if (!fast) {
                own_edges[0] = load_edge_cache(v, own.rp[0], own.rp[1], own.rp[P == 1 ? 1 : 2]);
                if constexpr (P == 4) own_edges[1] = load_edge_cache(v, own.rp[2], own.rp[3], own.rp[4]);
            }
        }
    }
    // TApSA windows of a fast run in LDS: in at the start, out at the end
    const bool lds_ring = fast && ring_res > 0;
    if (lds_ring) {
        const int32_t al = a.alpha;
        const size_t g0 = static_cast<size_t>(q >> 2) * n4 * al;
        for (int32_t x = threadIdx.x; x < n4 * al; x += BLOCK) lring[x] = a.ring[(g0 + x) * 4 + (q & 3)];
        __syncthreads();
    }
    if constexpr (kFastKind) {
        if (fast) {
            // slot chunks the wavefront needs: the largest row-pair length of
            // its lanes (every lane of the wavefront takes part)
            int32_t cnt = owns ? min(own.rp[P] - own.rp[0], fast_slots<P>()) : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) cnt = max(cnt, __shfl_xor(cnt, off));
            own_fast.chunks = static_cast<uint32_t>(
                __builtin_amdgcn_readfirstlane((cnt + fast_chunk<P>() - 1) / fast_chunk<P>()));
        }
    }
    // Fast layout, one step: read the buffer at offset RO, write all four
    // copies into the other.
    auto fast_step = [&](auto alg_tag, auto par_tag, auto lring_tag, uint32_t tau, float i0t, uint32_t k0,
                         uint32_t k1) __attribute__((always_inline)) {
        constexpr int ALG = decltype(alg_tag)::value;
        constexpr int PAR = decltype(par_tag)::value;
        constexpr bool LR = decltype(lring_tag)::value;
        constexpr uint32_t RO = PAR ? static_cast<uint32_t>(kFastStride) : 0u;
        constexpr uint32_t WO = PAR ? 0u : static_cast<uint32_t>(kFastStride);
        const uint32_t b = task_one_trial<CSR, LPT, ALG, !CSR_LDS, PAR ? kFieldFast1 : kFieldFast0, LR>(
            v, own, nullptr, &own_fast, &own_in, lring, sub, static_cast<uint32_t>(q), tau, i0t, smem + RO,
            k0, k1, st);
        unsigned char *to = smem + WO + own.base;
        if constexpr (P == 2) {
            const uint32_t m = b ^ 0x0101u;
            *reinterpret_cast<uint16_t *>(to) = static_cast<uint16_t>(b);
            *reinterpret_cast<uint16_t *>(to + n4) = static_cast<uint16_t>(m);
            *reinterpret_cast<uint16_t *>(to + 2 * n4) = static_cast<uint16_t>(b << 6);
            *reinterpret_cast<uint16_t *>(to + 3 * n4) = static_cast<uint16_t>(m << 6);
        } else {
            const uint32_t m = b ^ 1u;
            to[0] = static_cast<unsigned char>(b);
            to[n4] = static_cast<unsigned char>(m);
            to[2 * n4] = static_cast<unsigned char>(b << 6);
            to[3 * n4] = static_cast<unsigned char>(m << 6);
        }
    };
    // the step loop, instantiated per input stage (pSA, SpSA, TApSA) so that
    // plain pSA carries no per-update test for the others
    auto sweep = [&](auto alg_tag) {
    constexpr int ALG = decltype(alg_tag)::value;
    // period mode: t_res sub-steps per step (the counter of the random words
    // and of the period gate is the sub-step); otherwise one
    const int32_t nsub = ALG == kAlgPeriod ? a.t_res : 1;
    if constexpr (kFastKind) {
        if (fast) {
            // two steps per iteration: buffer 0 -> 1, then 1 -> 0
            auto run_fast = [&](auto lring_tag) __attribute__((always_inline)) {
                int32_t t = a.t_begin, s = 0, left = (a.t_end - a.t_begin) * nsub;
                auto half = [&](auto par_tag) __attribute__((always_inline)) {
                    const float i0t = a.i0[t];
                    uint32_t k0 = a.k0, k1 = a.k1;
                    asm volatile("" : "+s"(k0), "+s"(k1));
                    const uint32_t tau = static_cast<uint32_t>(t) * static_cast<uint32_t>(nsub) +
                                         static_cast<uint32_t>(s);
                    if (owns) fast_step(alg_tag, par_tag, lring_tag, tau, i0t, k0, k1);
                    __syncthreads();
                    if (++s == nsub) {
                        s = 0;
                        ++t;
                    }
                    --left;
                };
                bool in1 = false;
                while (left > 0) {
                    half(std::integral_constant<int, 0>{});
                    if (left == 0) {
                        in1 = true;
                        break;
                    }
                    half(std::integral_constant<int, 1>{});
                }
                cur = in1 ? buf1 : buf0;
                nxt = in1 ? buf0 : buf1;
            };
            if (ALG == kAlgTapsa && lds_ring)
                run_fast(std::true_type{});
            else
                run_fast(std::false_type{});
            return;
        }
    }
    for (int32_t t = a.t_begin; t < a.t_end; ++t) {
        const float i0t = a.i0[t];
        // the key, opaque to the optimiser at every step: the Philox key
        // schedule is then formed on the scalar unit where it is used rather
        // than hoisted out of the loop into registers that spill
        uint32_t k0 = a.k0, k1 = a.k1;
        asm volatile("" : "+s"(k0), "+s"(k1));
        for (int32_t s = 0; s < nsub; ++s) {
        const uint32_t tau = static_cast<uint32_t>(t) * static_cast<uint32_t>(nsub) + static_cast<uint32_t>(s);
        if constexpr (TPW == 1) {
            if (resident) {
                if (owns)
                    one_trial_step(alg_tag, std::true_type{}, own, own_edges, &own_in, tau, i0t, k0, k1, cur, nxt);
            } else {
                // the LPT lanes of a task share its slot, so they enter and leave together
                for (int32_t slot = threadIdx.x / LPT; slot < tasks; slot += BLOCK / LPT)
                    one_trial_step(alg_tag, std::false_type{}, load_task<LPT>(v, v.order[slot], sub),
                                   nullptr, nullptr, tau, i0t, k0, k1, cur, nxt);
            }
        } else {
            for (int32_t slot = threadIdx.x; slot < tasks; slot += BLOCK)
                task_four_trials<CSR, ALG, !CSR_LDS>(v, v.order[slot], q, tau, i0t,
                                      reinterpret_cast<const uint32_t *>(cur),
                                      reinterpret_cast<uint32_t *>(nxt), k0, k1, st);
        }
        __syncthreads();
        unsigned char *tmp = cur;
        cur = nxt;
        nxt = tmp;
        }
    }
    };
    if (a.t_res > 0)
        sweep(std::integral_constant<int, kAlgPeriod>{});
    else if (a.ring != nullptr)
        sweep(std::integral_constant<int, kAlgTapsa>{});
    else if (a.xs != nullptr)
        sweep(std::integral_constant<int, kAlgSpsa>{});
    else
        sweep(std::integral_constant<int, kAlgPsa>{});

    if constexpr (TPW == 1) {
        if (lds_ring) {
            const int32_t al = a.alpha;
            const size_t g0 = static_cast<size_t>(q >> 2) * n4 * al;
            for (int32_t x = threadIdx.x; x < n4 * al; x += BLOCK) a.ring[(g0 + x) * 4 + (q & 3)] = lring[x];
        }
        if (owns && a.xs != nullptr) {
            const size_t row0 = static_cast<size_t>(q >> 2) * n4 + own.base;
#pragma unroll
            for (int j = 0; j < P; ++j) a.xs[(row0 + j) * 4 + (q & 3)] = own_in.held[j];
        }
        for (int32_t i = threadIdx.x; i < n; i += BLOCK) {
            int8_t s;
            if constexpr (E::kU)
                s = cur[i] ? int8_t(1) : int8_t(-1);
            else
                s = static_cast<int8_t>(cur[i]);
            a.spins[static_cast<size_t>(i) * a.t4 + q] = s;
        }
    } else {
        const uint32_t *s = reinterpret_cast<const uint32_t *>(cur);
        for (int32_t i = threadIdx.x; i < n; i += BLOCK) {
            uint32_t w = s[i];
            if constexpr (E::kU) w = ((w ^ 0x01010101u) * 0xFEu) ^ 0x01010101u;
            *reinterpret_cast<uint32_t *>(a.spins + static_cast<size_t>(i) * a.t4 + 4 * q) = w;
        }
    }
}

template <int TPW, int LPT, int CSR, bool CSR_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void anneal_kernel(AnnealArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    anneal_body<TPW, LPT, CSR, CSR_LDS, BLOCK>(a, static_cast<int32_t>(blockIdx.x), smem);
}

// ---------------------------------------------------------------------------
// Batched launch: one grid over the work items of many runs.  Work item b is
// (run jobs[work[b].x], trial group work[b].y); each run carries its own
// graph, factors, spins and step range, and names its kernel variant.  All
// variants share one launch (dynamic LDS = the largest any item needs).
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void anneal_batch_kernel(const BatchJob *__restrict__ jobs,
                                                             const int2 *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 w = work[blockIdx.x];
    if (w.x < 0) return;  // padding slot of the XCD-aware work list
    const BatchJob &job = jobs[w.x];
    const AnnealArgs a = job.a;
    switch (job.variant) {
        case kBatchUnitLds2: anneal_body<1, 2, kCsrUnit, true, BLOCK>(a, w.y, smem); break;
        case kBatchUnitGlb2: anneal_body<1, 2, kCsrUnit, false, BLOCK>(a, w.y, smem); break;
        case kBatchUnitLds4: anneal_body<1, 4, kCsrUnit, true, BLOCK>(a, w.y, smem); break;
        case kBatchUnitGlb4: anneal_body<1, 4, kCsrUnit, false, BLOCK>(a, w.y, smem); break;
        case kBatchP32Lds2: anneal_body<1, 2, kCsrPack32, true, BLOCK>(a, w.y, smem); break;
        case kBatchP32Glb2: anneal_body<1, 2, kCsrPack32, false, BLOCK>(a, w.y, smem); break;
        case kBatchPairGlb2: anneal_body<1, 2, kCsrPair, false, BLOCK>(a, w.y, smem); break;
        case kBatchP16Lds4T: anneal_body<4, 1, kCsrPack16, true, BLOCK>(a, w.y, smem); break;
        case kBatchP16Glb4T: anneal_body<4, 1, kCsrPack16, false, BLOCK>(a, w.y, smem); break;
        case kBatchP32Lds4T: anneal_body<4, 1, kCsrPack32, true, BLOCK>(a, w.y, smem); break;
        case kBatchP32Glb4T: anneal_body<4, 1, kCsrPack32, false, BLOCK>(a, w.y, smem); break;
        case kBatchPairGlb4T: anneal_body<4, 1, kCsrPair, false, BLOCK>(a, w.y, smem); break;
        default: break;
    }
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

template <int LPT>
hipError_t launch_one_trial(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    switch (plan.csr) {
        case kCsrPair: return launch_lds<1, LPT, kCsrPair>(stream, args, plan);
        case kCsrPack32: return launch_lds<1, LPT, kCsrPack32>(stream, args, plan);
        case kCsrUnit: return launch_lds<1, LPT, kCsrUnit>(stream, args, plan);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_four_trials(hipStream_t stream, const AnnealArgs &args, const AnnealPlan &plan) {
    switch (plan.csr) {
        case kCsrPair: return launch_lds<4, 1, kCsrPair>(stream, args, plan);
        case kCsrPack32: return launch_lds<4, 1, kCsrPack32>(stream, args, plan);
        case kCsrPack16: return launch_lds<4, 1, kCsrPack16>(stream, args, plan);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool plan_anneal(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                 int32_t block_req, size_t max_lds, int32_t num_cu, AnnealPlan *plan,
                 std::string *why) {
    AnnealPlan p;
    const int32_t n4 = g.n4;
    const int32_t tasks = n4 / 4;
    if (tpw_req == 1 || tpw_req == 4) {
        p.tpw = tpw_req;
    } else {
        // four trials per workgroup share each CSR walk; one trial per
        // workgroup exposes four times the workgroups
        p.tpw = (run.t4 / 4 >= num_cu) ? 4 : 1;
    }
    p.grid = p.tpw == 4 ? run.t4 / 4 : run.trials;
    if (p.tpw == 4) {
        p.csr = (g.pk16 && g.max_degree <= 255) ? kCsrPack16 : (g.pk32 ? kCsrPack32 : kCsrPair);
        p.lpt = 1;
    } else {
        p.csr = g.ux16 ? kCsrUnit : (g.pk32 ? kCsrPack32 : kCsrPair);
        if (lpt_req == 1 || lpt_req == 2 || lpt_req == 4)
            p.lpt = lpt_req;
        else  // spread tasks over more lanes while the workgroup has lanes to spare
            p.lpt = tasks * 4 <= 1024 ? 4 : (tasks * 2 <= 1024 ? 2 : 1);
    }
    const size_t sp = 2 * spin_stride(n4, p.tpw, p.lpt, p.csr) +
                      ring_lds_bytes(n4, p.tpw, p.lpt, p.csr, run.ring != nullptr, run.alpha);
    if (sp > max_lds) {
        // four trials' spin state too large: one trial per workgroup if the
        // choice was the planner's
        if (p.tpw == 4 && tpw_req != 4)
            return plan_anneal(g, run, 1, lpt_req, block_req, max_lds, num_cu, plan, why);
        if (why)
            *why = "n = " + std::to_string(g.n) + " does not fit the LDS-resident spin state (" +
                   std::to_string(sp) + " > " + std::to_string(max_lds) + " bytes)";
        return false;
    }
    const size_t full = sp + params_bytes(n4) + align16(static_cast<size_t>(g.nnz) * edge_bytes(p.csr));
    p.csr_lds = full <= max_lds ? 1 : 0;
    p.lds_bytes = p.csr_lds ? full : sp;
    const int32_t lanes = tasks * p.lpt;
    if (block_req == 256 || block_req == 512 || block_req == 1024)
        p.block = block_req;
    else
        p.block = lanes > 512 ? 1024 : (lanes > 256 ? 512 : 256);
    *plan = p;
    return true;
}

void task_order(const DevGraph &g, const std::vector<int32_t> &row_ptr_host, const AnnealPlan &plan,
                std::vector<int32_t> *order) {
    const int32_t tasks = g.n4 / 4;
    std::vector<int64_t> key(static_cast<size_t>(tasks));
    for (int32_t m = 0; m < tasks; ++m) {
        int64_t d[4];
        for (int p = 0; p < 4; ++p) d[p] = row_ptr_host[4 * m + p + 1] - row_ptr_host[4 * m + p];
        if (plan.tpw == 1 && plan.lpt == 2)
            key[m] = std::max(d[0] + d[1], d[2] + d[3]);
        else if (plan.tpw == 1 && plan.lpt == 4)
            key[m] = std::max(std::max(d[0], d[1]), std::max(d[2], d[3]));
        else
            key[m] = d[0] + d[1] + d[2] + d[3];
    }
    order->resize(static_cast<size_t>(tasks));
    for (int32_t m = 0; m < tasks; ++m) (*order)[m] = m;
    // heaviest tasks first: lanes of a wavefront walk rows of similar length
    std::stable_sort(order->begin(), order->end(),
                     [&](int32_t x, int32_t y) { return key[x] > key[y]; });
}

// LDS the kernel carves for a run under a plan (the layout above).
size_t lds_need(const DevGraph &g, const DevRun &run, const AnnealPlan &p) {
    size_t b = 2 * spin_stride(g.n4, p.tpw, p.lpt, p.csr) +
               ring_lds_bytes(g.n4, p.tpw, p.lpt, p.csr, run.ring != nullptr, run.alpha);
    if (p.csr_lds) b += params_bytes(g.n4) + align16(static_cast<size_t>(g.nnz) * edge_bytes(p.csr));
    return b;
}

hipError_t launch_anneal(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const AnnealPlan &plan, const int32_t *order, int32_t t_begin,
                         int32_t t_end) {
    if (t_end <= t_begin) return hipSuccess;
    // a plan made for another input stage would leave the kernel's LDS
    // layout outside the allocation
    if (lds_need(g, run, plan) > plan.lds_bytes) return hipErrorInvalidValue;
    // the four-trial sweep over rows in device memory reads the ELL rows
    if (plan.tpw == 4 && plan.csr == kCsrPack16 && !plan.csr_lds && (!g.ell || !run.pp))
        return hipErrorInvalidValue;
    AnnealArgs a;
    fill_anneal_args(&a, g, run, order, t_begin, t_end);
    if (plan.tpw == 4) return launch_four_trials(stream, a, plan);
    switch (plan.lpt) {
        case 1: return launch_one_trial<1>(stream, a, plan);
        case 2: return launch_one_trial<2>(stream, a, plan);
        case 4: return launch_one_trial<4>(stream, a, plan);
        default: return hipErrorInvalidValue;
    }
}

void fill_anneal_args(AnnealArgs *a, const DevGraph &g, const DevRun &run, const int32_t *order,
                      int32_t t_begin, int32_t t_end) {
    a->n = g.n;
    a->n4 = g.n4;
    a->t4 = run.t4;
    a->t_begin = t_begin;
    a->t_end = t_end;
    a->nnz = static_cast<int32_t>(g.nnz);
    a->tasks = g.n4 / 4;
    a->row_ptr = g.row_ptr;
    a->col = g.col;
    a->val = g.val;
    a->pk32 = g.pk32;
    a->pk16 = g.pk16;
    a->ux16 = g.ux16;
    a->ell = g.ell;
    a->eptr = g.eptr;
    a->pp = run.pp;
    a->h = g.h;
    a->i0 = run.i0;
    a->lam = run.lambda;
    a->dlt = run.delta;
    a->thr = run.thr24;
    a->order = order;
    a->k0 = run.key0;
    a->k1 = run.key1;
    a->spins = run.spins;
    a->xs = run.xs;
    a->stall24 = run.stall24;
    a->ring = run.ring;
    a->alpha = run.alpha;
    a->t_res = run.t_res;
}

bool plan_batch_item(const DevGraph &g, const DevRun &run, int32_t tpw_req, int32_t lpt_req,
                     size_t max_lds, AnnealPlan *plan, int32_t *variant, std::string *why) {
    AnnealPlan p;
    if (tpw_req == 4) {
        if (!plan_anneal(g, run, 4, 1, 0, max_lds, 1 << 30, &p, why)) return false;
        if (p.csr == kCsrPack16) {
            if (!p.csr_lds && (!g.ell || !run.pp)) {
                if (why) *why = "four-trial run without its ELL rows";
                return false;
            }
            *variant = p.csr_lds ? kBatchP16Lds4T : kBatchP16Glb4T;
        } else if (p.csr == kCsrPack32) {
            *variant = p.csr_lds ? kBatchP32Lds4T : kBatchP32Glb4T;
        } else {
            *variant = kBatchPairGlb4T;
            p.csr_lds = 0;
            p.lds_bytes = 2 * spin_buf_bytes(g.n4, 4, kCsrPair);
        }
        *plan = p;
        return true;
    }
    if (!plan_anneal(g, run, 1, lpt_req == 4 ? 4 : 2, 0, max_lds, 1 << 30, &p, why)) return false;
    if (p.csr == kCsrUnit) {
        *variant = p.lpt == 4 ? (p.csr_lds ? kBatchUnitLds4 : kBatchUnitGlb4)
                              : (p.csr_lds ? kBatchUnitLds2 : kBatchUnitGlb2);
    } else {
        p.lpt = 2;
        if (p.csr == kCsrPack32) {
            *variant = p.csr_lds ? kBatchP32Lds2 : kBatchP32Glb2;
        } else {
            *variant = kBatchPairGlb2;
            p.csr_lds = 0;
            p.lds_bytes = 2 * spin_buf_bytes(g.n4, 1, kCsrPair);
        }
    }
    *plan = p;
    return true;
}

hipError_t launch_anneal_batch(hipStream_t stream, const BatchJob *jobs, const int2 *work,
                               int32_t nwork, int32_t block, size_t lds_bytes) {
    if (nwork <= 0) return hipSuccess;
    const void *kern;
    switch (block) {
        case 256: kern = reinterpret_cast<const void *>(anneal_batch_kernel<256>); break;
        case 512: kern = reinterpret_cast<const void *>(anneal_batch_kernel<512>); break;
        case 1024: kern = reinterpret_cast<const void *>(anneal_batch_kernel<1024>); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t err = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds_bytes));
    if (err != hipSuccess) return err;
    switch (block) {
        case 256:
            hipLaunchKernelGGL(anneal_batch_kernel<256>, dim3(nwork), dim3(256), lds_bytes, stream, jobs, work);
            break;
        case 512:
            hipLaunchKernelGGL(anneal_batch_kernel<512>, dim3(nwork), dim3(512), lds_bytes, stream, jobs, work);
            break;
        default:
            hipLaunchKernelGGL(anneal_batch_kernel<1024>, dim3(nwork), dim3(1024), lds_bytes, stream, jobs, work);
            break;
    }
    return hipGetLastError();
}

}  // namespace psa
