// period.hip -- the sweep of period-mode timing (Eq. 6's timing factor as
// integer periods; the listing's count mod nu gate), one trial per workgroup.
//
// A cycle (one step of the schedule) has t_res sub-steps tau = t t_res + s.
// At sub-step tau every p-bit whose period divides tau updates from the
// spins of sub-step tau - 1 (synchronously, I0 of cycle t, r from the Philox
// word i mod 4 of counter (tau, i/4, k, 1)); the others hold.  With periods
// near t_res only about one p-bit in t_res fires per sub-step, and the fired
// p-bits are scattered, so a sweep over all p-bits per sub-step would run the
// whole update path in nearly every wavefront.  Here the p-bits are sorted
// by period into classes (contiguous ranges of a per-position record list);
// each wavefront keeps one countdown per class (lane c for class c), so a
// sub-step knows with one ballot which classes fire, and only their p-bits
// are visited.  Sub-steps where nothing fires cost a few scalar instructions.
//
// Spins: one LDS buffer of int8 +-1, updated in place in two phases per
// firing sub-step: every fired p-bit's new value is computed from the buffer
// (a lane keeps its first two in registers and stages the rest in LDS by
// sorted position), a barrier, the new values are written, a barrier.  The
// neighbour terms of a row are read in straight-line chunks of eight edges
// (clamped addresses, zero couplings past the row's end), so a row costs two
// LDS round trips per chunk rather than two per edge.
//
// Graphs of up to 2,048 p-bits with 16-bit edge words take resident lanes
// instead: lane l of a B-lane workgroup owns the sorted positions s B + l
// (slots s < K, K = 1, 2, 4 or 8 p-bits) for the whole launch, with their records and their rows'
// first edge words in registers.  A sub-step then costs a firing lane one LDS
// round trip for the neighbours' spins (more only past the cached edges) and
// the decision, and a wavefront whose p-bits do not fire only the two
// barriers.  A wavefront's slot holds 64 consecutive positions in period
// order, so they mostly share a period and fire together, and a class's
// positions spread over consecutive wavefronts, hence over the four SIMDs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {

namespace {

constexpr size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

struct PeriodArgs {
    int32_t n, t4, t_begin, t_end, t_res, nclass;
    int32_t sbuf;           // bytes per LDS spin buffer
    int32_t nnz;
    const PeriodRec *recs;  // [n] by class
    const PeriodClass *classes;
    const uint32_t *pk32;   // edges as col | J << 16, or nullptr
    const int32_t *col;
    const int32_t *val;
    const float *i0;
    uint32_t k0, k1;
    int8_t *spins;          // [n][t4]
};

// Eight neighbour terms of a row from edge x0 on: couplings times the
// neighbours' spins, addresses clamped to the edge before rp1 (edge 0 for an
// empty first row; the graph has an edge) and couplings zero past the end.
// `between` runs after the edge words are requested and before the spins are
// (work that hides the first load's latency), `after` once the spin loads
// are in flight.
template <bool PK32, typename F, typename G>
__device__ __forceinline__ int32_t chunk_field(int32_t x0, int32_t rp1, const uint32_t *pk,
                                               const int32_t *col, const int32_t *val, const int8_t *s,
                                               F &&between, G &&after) {
    constexpr int kC = 8;
    int32_t j[kC], J[kC], m[kC];
    uint32_t w[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
        const bool in = x0 + u < rp1;
        const int32_t x = in ? x0 + u : (rp1 > 0 ? rp1 - 1 : 0);
        if constexpr (PK32) {
            w[u] = pk[x];
        } else {
            j[u] = col[x];
            J[u] = val[x];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    between();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kC; ++u) {
        const bool in = x0 + u < rp1;
        if constexpr (PK32) {
            j[u] = static_cast<int32_t>(w[u] & 0xFFFFu);
            J[u] = in ? static_cast<int32_t>(w[u]) >> 16 : 0;
        } else {
            J[u] = in ? J[u] : 0;
        }
        m[u] = s[j[u]];
    }
    __builtin_amdgcn_sched_barrier(0);
    after();
    __builtin_amdgcn_sched_barrier(0);
    int32_t L = 0;
#pragma unroll
    for (int u = 0; u < kC; ++u) L += J[u] * m[u];
    return L;
}

template <bool IN_LDS, bool PK32, int BLOCK>
__global__ __launch_bounds__(BLOCK) void period_kernel(PeriodArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t q = static_cast<int32_t>(blockIdx.x);  // trial
    const int tid = static_cast<int>(threadIdx.x);
    const int lane = tid & 63;
    const int32_t n = a.n;
    int8_t *spin = reinterpret_cast<int8_t *>(smem);
    int8_t *staged = spin + a.sbuf;  // new values past a lane's first two, by position
    const PeriodRec *recs = a.recs;
    const uint32_t *pk = a.pk32;
    const int32_t *col = a.col;
    const int32_t *val = a.val;
    if constexpr (IN_LDS) {
        PeriodRec *lrec = reinterpret_cast<PeriodRec *>(smem + 2 * static_cast<size_t>(a.sbuf));
        const int4 *src = reinterpret_cast<const int4 *>(a.recs);
        int4 *dst = reinterpret_cast<int4 *>(lrec);
        for (int32_t x = tid; x < 2 * n; x += BLOCK) dst[x] = src[x];
        unsigned char *e = smem + 2 * static_cast<size_t>(a.sbuf) + al16(sizeof(PeriodRec) * static_cast<size_t>(n));
        if constexpr (PK32) {
            uint32_t *le = reinterpret_cast<uint32_t *>(e);
            for (int32_t x = tid; x < a.nnz; x += BLOCK) le[x] = a.pk32[x];
            pk = le;
        } else {
            int32_t *lc = reinterpret_cast<int32_t *>(e);
            int32_t *lv = lc + a.nnz;
            for (int32_t x = tid; x < a.nnz; x += BLOCK) {
                lc[x] = a.col[x];
                lv[x] = a.val[x];
            }
            col = lc;
            val = lv;
        }
        recs = lrec;
    }
    for (int32_t i = tid; i < n; i += BLOCK) spin[i] = a.spins[static_cast<size_t>(i) * a.t4 + q];
    // lane c of every wavefront carries class c: period, range, countdown
    // (tau mod period); every wavefront computes the same masks
    const uint32_t tau0 = static_cast<uint32_t>(a.t_begin) * static_cast<uint32_t>(a.t_res);
    const uint32_t tau_end = static_cast<uint32_t>(a.t_end) * static_cast<uint32_t>(a.t_res);
    const bool has = lane < a.nclass;
    uint32_t per = 1u, cnt = 1u;
    int32_t cb = 0, ce = 0;
    if (has) {
        const PeriodClass c = a.classes[lane];
        per = c.period;
        cb = c.begin;
        ce = c.end;
        cnt = tau0 % per;
    }
    __syncthreads();
    const uint32_t k0 = a.k0, k1 = a.k1;
    const uint32_t kq = static_cast<uint32_t>(q);
    int32_t t = a.t_begin, s = 0;
    float i0t = a.i0[t];
    // the next cycle's I0, loaded a cycle ahead of its use
    float i0n = t + 1 < a.t_end ? a.i0[t + 1] : 0.0f;
    for (uint32_t tau = tau0; tau < tau_end; ++tau) {
        const uint64_t fire = __ballot(has && cnt == 0u);
        cnt = (cnt + 1u == per) ? 0u : cnt + 1u;
        if (fire != 0u) {
            // phase 1: new values of the fired p-bits from the current spins
            int32_t ia = -1, ib = -1;
            int8_t va = 0, vb = 0;
            int32_t done = 0;
            uint64_t m = fire;
            uint32_t off = 0;
            while (m != 0u) {
                const int c = __builtin_ctzll(m);
                m &= m - 1u;
                const int32_t b = __builtin_amdgcn_readlane(cb, c);
                const int32_t e = __builtin_amdgcn_readlane(ce, c);
                const int32_t first = static_cast<int32_t>((static_cast<uint32_t>(tid) - off) & (BLOCK - 1));
                for (int32_t idx = b + first; idx < e; idx += BLOCK) {
                    const PeriodRec r = recs[idx];
                    // the first eight edges, with the random block's rounds
                    // placed under their two load latencies
                    PhiloxState ps = philox_start(tau, static_cast<uint32_t>(r.i) >> 2, kq, kTagR, k0, k1);
                    auto half = [&]() {
                        philox_rounds<5>(ps);
                        // pinned here (not sunk to the decision after the loop)
                        asm volatile("" : "+v"(ps.c0), "+v"(ps.c1), "+v"(ps.c2), "+v"(ps.c3));
                    };
                    int32_t L = chunk_field<PK32>(r.rp0, r.rp1, pk, col, val, spin, half, half);
                    const Words4 w4{ps.c0, ps.c1, ps.c2, ps.c3};
                    for (int32_t x0 = r.rp0 + 8; x0 < r.rp1; x0 += 8)
                        L += chunk_field<PK32>(x0, r.rp1, pk, col, val, spin, []() {}, []() {});
                    L += r.h;
                    const float xin = (i0t * r.lam) * (static_cast<float>(L) + r.dlt);
                    const uint32_t word = word_of(w4, static_cast<uint32_t>(r.i) & 3u);
                    const int8_t v = pbit_up(xin, word) ? int8_t(1) : int8_t(-1);
                    if (done == 0) {
                        ia = r.i;
                        va = v;
                    } else if (done == 1) {
                        ib = r.i;
                        vb = v;
                    } else {
                        staged[idx] = v;
                    }
                    ++done;
                }
                off = (off + static_cast<uint32_t>(e - b)) & (BLOCK - 1);
            }
            __syncthreads();
            // phase 2: write them
            if (ia >= 0) spin[ia] = va;
            if (ib >= 0) spin[ib] = vb;
            if (done > 2) {
                // this lane's positions past its first two, in the same order
                int32_t seen = 0;
                m = fire;
                off = 0;
                while (m != 0u) {
                    const int c = __builtin_ctzll(m);
                    m &= m - 1u;
                    const int32_t b = __builtin_amdgcn_readlane(cb, c);
                    const int32_t e = __builtin_amdgcn_readlane(ce, c);
                    const int32_t first = static_cast<int32_t>((static_cast<uint32_t>(tid) - off) & (BLOCK - 1));
                    for (int32_t idx = b + first; idx < e; idx += BLOCK) {
                        if (seen >= 2) spin[recs[idx].i] = staged[idx];
                        ++seen;
                    }
                    off = (off + static_cast<uint32_t>(e - b)) & (BLOCK - 1);
                }
            }
            __syncthreads();
        }
        if (++s == a.t_res) {
            s = 0;
            ++t;
            i0t = i0n;
            if (t + 1 < a.t_end) i0n = a.i0[t + 1];
        }
    }
    for (int32_t i = tid; i < n; i += BLOCK) a.spins[static_cast<size_t>(i) * a.t4 + q] = spin[i];
}

// Resident lanes: K p-bits per lane, C edge words of each cached.  Spins in
// two regions kResStride bytes apart (read one, write the other, one barrier
// per firing sub-step); with unit couplings (UNIT) each region holds the
// spins and, kResNeg bytes on, their negations, and a cached edge is the
// byte offset of the neighbour's spin or of its negation, so the neighbour
// term is a plain sum of loads.  Otherwise a cached edge is col | J << 16.
constexpr int32_t kResMaxN = 2048;    // p-bits on resident lanes at most
constexpr int32_t kResZero = kResMaxN;          // a zero byte past the spins
constexpr int32_t kResNeg = kResMaxN + 16;      // the negations
constexpr int32_t kResStride = 2 * kResMaxN + 16;  // one region: spins, zero, negations
constexpr int32_t kResEdges = 2 * kResStride;  // edges past the caches, in LDS
constexpr int32_t kResDefaultBlock = 1024;

template <int K, int C, bool IN_LDS, bool UNIT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void period_resident_kernel(PeriodArgs a, const uint32_t *ecache) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t q = static_cast<int32_t>(blockIdx.x);  // trial
    const int tid = static_cast<int>(threadIdx.x);
    const int lane = tid & 63;
    const int32_t n = a.n;
    const uint32_t *pk = a.pk32;
    if constexpr (IN_LDS) {
        uint32_t *le = reinterpret_cast<uint32_t *>(smem + kResEdges);
        for (int32_t x = tid; x < a.nnz; x += BLOCK) le[x] = a.pk32[x];
        pk = le;
    }
    // the lane's p-bits: record fields, cached edges, current spins
    int32_t oi[K], orp[K], oend[K], oh[K], ocls[K];
    float olam[K], odlt[K];
    uint32_t oc[K][C];
    int8_t cv[K];
    // the random word of each p-bit's next firing sub-step nt, drawn ahead
    // (it does not depend on the spins): after a p-bit fires, its word for
    // the sub-step one period later is drawn at the next firing sub-step,
    // off the firing p-bits' path
    uint32_t oper[K], nt[K], nw[K];
    bool pend[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int32_t pos = s * BLOCK + tid;
        cv[s] = 1;
        oper[s] = 1u;
        pend[s] = false;
        if (pos < n) {
            const PeriodRec r = a.recs[pos];
            oi[s] = r.i;
            orp[s] = r.rp0 + C;
            oend[s] = r.rp1;
            oh[s] = r.h;
            olam[s] = r.lam;
            odlt[s] = r.dlt;
            ocls[s] = r.cls;
#pragma unroll
            for (int u = 0; u < C; ++u) oc[s][u] = ecache[static_cast<size_t>(pos) * C + u];
            cv[s] = a.spins[static_cast<size_t>(r.i) * a.t4 + q];
        } else {
            oi[s] = 0;
            orp[s] = oend[s] = 0;
            oh[s] = 0;
            olam[s] = odlt[s] = 0.0f;
            ocls[s] = kPeriodMaxClasses;  // never fires
#pragma unroll
            for (int u = 0; u < C; ++u) oc[s][u] = UNIT ? static_cast<uint32_t>(kResZero) : 0u;
        }
    }
    int8_t *spin = reinterpret_cast<int8_t *>(smem);
    for (int32_t i = tid; i < n; i += BLOCK) {
        const int8_t v = a.spins[static_cast<size_t>(i) * a.t4 + q];
        spin[i] = v;
        spin[kResStride + i] = v;
        if constexpr (UNIT) {
            spin[kResNeg + i] = static_cast<int8_t>(-v);
            spin[kResStride + kResNeg + i] = static_cast<int8_t>(-v);
        }
    }
    if constexpr (UNIT) {
        // the padding entry of unused cache slots: a zero byte
        if (tid == 0) {
            spin[kResZero] = 0;
            spin[kResStride + kResZero] = 0;
        }
    }
    const uint32_t tau0 = static_cast<uint32_t>(a.t_begin) * static_cast<uint32_t>(a.t_res);
    const bool has = lane < a.nclass;
    uint32_t per = 1u, cnt = 1u;
    if (has) {
        per = a.classes[lane].period;
        cnt = tau0 % per;
    }
    const uint32_t k0 = a.k0, k1 = a.k1;
    const uint32_t kq = static_cast<uint32_t>(q);
    auto word_at = [&](uint32_t tau, int32_t i) __attribute__((always_inline)) {
        return word_of(philox4x32_10(tau, static_cast<uint32_t>(i) >> 2, kq, kTagR, k0, k1),
                       static_cast<uint32_t>(i) & 3u);
    };
#pragma unroll
    for (int s = 0; s < K; ++s) {
        nt[s] = 0u;
        nw[s] = 0u;
        if (ocls[s] < kPeriodMaxClasses) {
            oper[s] = a.classes[ocls[s]].period;
            nt[s] = tau0 + (oper[s] - tau0 % oper[s]) % oper[s];  // first firing
            nw[s] = word_at(nt[s], oi[s]);
        }
    }
    // the classes of this wavefront's p-bits: each slot holds 64 consecutive
    // positions in class order, so a range from its first lane's class to
    // its last valid lane's
    uint64_t wmask = 0;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int32_t lo = __builtin_amdgcn_readfirstlane(ocls[s]);
        const int32_t base = s * BLOCK + (tid & ~63);
        const int32_t last = min(63, n - 1 - base);
        if (last >= 0) {
            const int32_t hi = __builtin_amdgcn_readlane(ocls[s], last);
            const uint64_t upto = hi >= 63 ? ~0ull : ((2ull << hi) - 1ull);
            wmask |= upto & ~((1ull << lo) - 1ull);
        }
    }
    // the mask is the same in every lane (built from lane reads of the
    // wavefront's own slots); read it back through the scalar unit so that
    // the per-sub-step test below is a scalar branch, not a divergent one
    // with the execution mask saved and merged around the barrier
    wmask = (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(wmask >> 32))) << 32) |
            static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(wmask)));
    __syncthreads();
    uint64_t prev = 0;  // the classes of the previous firing sub-step
    bool pf[K];
#pragma unroll
    for (int s = 0; s < K; ++s) pf[s] = false;
    // one firing sub-step reading region PAR and writing the other
    auto firing = [&](auto par_tag, uint64_t fire, uint32_t tau, float i0t) __attribute__((always_inline)) {
        constexpr int PAR = decltype(par_tag)::value;
        constexpr int32_t RO = PAR * kResStride, WO = (1 - PAR) * kResStride;
        bool f[K];
#pragma unroll
        for (int s = 0; s < K; ++s) f[s] = ocls[s] < kPeriodMaxClasses && ((fire >> ocls[s]) & 1u) != 0u;
        float xin[K];
        bool close = false;
        // the firing p-bits' cached neighbour loads first, so that their LDS
        // latency passes under the random blocks below
        int32_t m[K][C];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (f[s]) {
#pragma unroll
                for (int u = 0; u < C; ++u) {
                    if constexpr (UNIT)
                        m[s][u] = spin[oc[s][u] + RO];
                    else
                        m[s][u] = spin[(oc[s][u] & 0xFFFFu) + RO];
                }
            }
        }
        // words of the p-bits that fired at the previous firing sub-step, for
        // their next firing (before the decisions below: a p-bit firing again
        // now takes its word from here)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (pend[s]) {
                nt[s] += oper[s];
                nw[s] = word_at(nt[s], oi[s]);
                pend[s] = false;
            }
        }
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (f[s]) {
                int32_t L = oh[s];
#pragma unroll
                for (int u = 0; u < C; ++u) {
                    if constexpr (UNIT)
                        L += m[s][u];
                    else
                        L += (static_cast<int32_t>(oc[s][u]) >> 16) * m[s][u];
                }
                for (int32_t x0 = orp[s]; x0 < oend[s]; x0 += 8)
                    L += chunk_field<true>(x0, oend[s], pk, nullptr, nullptr, spin + RO, []() {}, []() {});
                xin[s] = (i0t * olam[s]) * (static_cast<float>(L) + odlt[s]);
                const float diff = tanh_estimate_minus(xin[s], r_of(nw[s]));
                close = close || !estimate_decides(diff);
                cv[s] = diff > 0.0f ? int8_t(1) : int8_t(-1);
                pend[s] = true;
            }
        }
        // decisions from the tanh estimate; when some lane of the wave holds
        // one within 2^-16 of r, the firing slots are retaken with the exact
        // recipe (one uniform branch per sub-step, none per p-bit)
        if (__ballot(close) != 0u) {
#pragma unroll
            for (int s = 0; s < K; ++s)
                if (f[s]) cv[s] = tanh_f32(xin[s]) > r_of(nw[s]) ? int8_t(1) : int8_t(-1);
        }
        // the written region lacks this sub-step's and the previous firing
        // sub-step's changes: both are in the lanes' registers
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (f[s] || pf[s]) {
                spin[WO + oi[s]] = cv[s];
                if constexpr (UNIT) spin[WO + kResNeg + oi[s]] = static_cast<int8_t>(-cv[s]);
            }
            pf[s] = f[s];
        }
        __syncthreads();
    };
    bool par = false;
    const uint32_t tau_end = static_cast<uint32_t>(a.t_end) * static_cast<uint32_t>(a.t_res);
    int32_t t = a.t_begin, st = 0;
    float i0t = a.i0[t];
    // the next cycle's I0, loaded a cycle ahead of its use
    float i0n = t + 1 < a.t_end ? a.i0[t + 1] : 0.0f;
    for (uint32_t tau = tau0; tau < tau_end; ++tau) {
        const uint64_t fire = __ballot(has && cnt == 0u);
        cnt = (cnt + 1u == per) ? 0u : cnt + 1u;
        if (fire != 0u) {
            // a wavefront none of whose p-bits fires now or fired at the
            // previous firing sub-step has nothing to write: the barrier only
            if (((fire | prev) & wmask) != 0u) {
                if (par)
                    firing(std::integral_constant<int, 1>{}, fire, tau, i0t);
                else
                    firing(std::integral_constant<int, 0>{}, fire, tau, i0t);
            } else {
                __syncthreads();
            }
            par = !par;
            prev = fire;
        }
        if (++st == a.t_res) {
            st = 0;
            ++t;
            i0t = i0n;
            if (t + 1 < a.t_end) i0n = a.i0[t + 1];
        }
    }
#pragma unroll
    for (int s = 0; s < K; ++s)
        if (s * BLOCK + tid < n) a.spins[static_cast<size_t>(oi[s]) * a.t4 + q] = cv[s];
}

template <int K, int C, int B, bool IN_LDS, bool UNIT>
hipError_t launch_resident(hipStream_t stream, const PeriodArgs &a, const PeriodPlan &p,
                           const uint32_t *ecache, int32_t grid) {
    auto kern = period_resident_kernel<K, C, IN_LDS, UNIT, B>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(p.lds_bytes));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(B), p.lds_bytes, stream, a, ecache);
    return hipGetLastError();
}

template <int K, int C, int B>
hipError_t launch_resident_k(hipStream_t stream, const PeriodArgs &a, const PeriodPlan &p,
                             const uint32_t *ecache, int32_t grid) {
    switch (p.in_lds * 2 + p.unit) {
        case 0: return launch_resident<K, C, B, false, false>(stream, a, p, ecache, grid);
        case 1: return launch_resident<K, C, B, false, true>(stream, a, p, ecache, grid);
        case 2: return launch_resident<K, C, B, true, false>(stream, a, p, ecache, grid);
        default: return launch_resident<K, C, B, true, true>(stream, a, p, ecache, grid);
    }
}

// Lanes and p-bits per lane of the resident sweep: (block, K) with K the
// fewest of 1, 2, 4, 8 that covers n (K <= 2 at 1,024 lanes and <= 4 at
// 512, whose registers are fewer); 0 if none.
int32_t resident_k_for(int32_t n, int32_t block) {
    const int32_t kmax = block == 1024 ? 2 : (block == 512 ? 4 : 8);
    for (int32_t k = 1; k <= kmax; k *= 2)
        if (static_cast<int64_t>(k) * block >= n) return k;
    return 0;
}

int32_t resident_cache(int32_t k) { return k == 1 ? 16 : (k <= 4 ? 12 : 8); }

template <bool IN_LDS, bool PK32>
hipError_t launch_block(hipStream_t stream, const PeriodArgs &a, const PeriodPlan &p, int32_t grid) {
    const void *kern;
    switch (p.block) {
        case 256: kern = reinterpret_cast<const void *>(period_kernel<IN_LDS, PK32, 256>); break;
        case 512: kern = reinterpret_cast<const void *>(period_kernel<IN_LDS, PK32, 512>); break;
        case 1024: kern = reinterpret_cast<const void *>(period_kernel<IN_LDS, PK32, 1024>); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t err = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(p.lds_bytes));
    if (err != hipSuccess) return err;
    if (p.block == 256)
        hipLaunchKernelGGL((period_kernel<IN_LDS, PK32, 256>), dim3(grid), dim3(256), p.lds_bytes, stream, a);
    else if (p.block == 512)
        hipLaunchKernelGGL((period_kernel<IN_LDS, PK32, 512>), dim3(grid), dim3(512), p.lds_bytes, stream, a);
    else
        hipLaunchKernelGGL((period_kernel<IN_LDS, PK32, 1024>), dim3(grid), dim3(1024), p.lds_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace

bool plan_period(const DevGraph &g, const DevRun &run, const std::vector<int32_t> &row_ptr_host,
                 const std::vector<int32_t> &col_host, const std::vector<int32_t> &val_host,
                 const std::vector<int32_t> &h_host, const std::vector<float> &lam,
                 const std::vector<float> &dlt, const std::vector<uint32_t> &periods, size_t max_lds,
                 int32_t block_req, PeriodPlan *plan, std::vector<PeriodRec> *recs,
                 std::vector<PeriodClass> *classes, std::vector<uint32_t> *ecache) {
    const int32_t n = g.n;
    // the sweep reads edge 0 for empty rows, so the graph needs an edge
    if (run.t_res < 1 || n < 1 || g.nnz < 1) return false;
    // classes: distinct periods in increasing order, members by index
    std::map<uint32_t, std::vector<int32_t>> by;
    for (int32_t i = 0; i < n; ++i) by[periods[i]].push_back(i);
    if (by.size() > static_cast<size_t>(kPeriodMaxClasses)) return false;
    PeriodPlan p;
    p.nclass = static_cast<int32_t>(by.size());
    p.pk32 = g.pk32 != nullptr ? 1 : 0;
    const size_t sbuf = al16(static_cast<size_t>(g.n4));
    p.sbuf = static_cast<int32_t>(sbuf);
    const size_t spins = 2 * sbuf;
    if (spins > max_lds) return false;
    const size_t full = spins + al16(sizeof(PeriodRec) * static_cast<size_t>(n)) +
                        static_cast<size_t>(g.nnz) * (p.pk32 ? 4 : 8);
    p.in_lds = full <= max_lds ? 1 : 0;
    p.lds_bytes = p.in_lds ? full : spins;
    // about one p-bit in t_res fires per sub-step, up to about three times
    // that where several classes fire together: a lane or two per p-bit
    const int32_t per_step = 2 * n / std::max(run.t_res, 1);
    p.block = per_step > 512 ? 1024 : (per_step > 256 ? 512 : 256);
    if (block_req == 256 || block_req == 512 || block_req == 1024) p.block = block_req;
    recs->clear();
    recs->reserve(static_cast<size_t>(n));
    classes->clear();
    ecache->clear();
    for (const auto &kv : by) {
        PeriodClass c{};
        c.period = kv.first;
        c.begin = static_cast<int32_t>(recs->size());
        for (int32_t i : kv.second) {
            PeriodRec r{};
            r.i = i;
            r.rp0 = row_ptr_host[i];
            r.rp1 = row_ptr_host[i + 1];
            r.h = h_host[i];
            r.lam = lam[i];
            r.dlt = dlt[i];
            r.cls = static_cast<int32_t>(classes->size());
            recs->push_back(r);
        }
        c.end = static_cast<int32_t>(recs->size());
        classes->push_back(c);
    }
    // resident lanes: 16-bit edge words (every |J| < 2^15), n <= 2,048; the
    // edge words past the cached ones in LDS when they fit.  Fewer lanes with
    // more p-bits each were measured slower (each lane's firing p-bits are
    // the sub-step's critical path)
    const int32_t rblock = (block_req == 256 || block_req == 512 || block_req == 1024) ? block_req
                                                                                        : kResDefaultBlock;
    const int32_t k = n <= kResMaxN ? resident_k_for(n, rblock) : 0;
    if (k > 0 && g.pk32 != nullptr) {
        p.resident_k = k;
        p.cache = resident_cache(k);
        p.block = rblock;
        p.unit = std::all_of(val_host.begin(), val_host.end(), [](int32_t v) { return v == 1 || v == -1; })
                     ? 1 : 0;
        const size_t rfull = static_cast<size_t>(kResEdges) + static_cast<size_t>(g.nnz) * 4;
        p.in_lds = rfull <= max_lds ? 1 : 0;
        p.lds_bytes = p.in_lds ? rfull : static_cast<size_t>(kResEdges);
        // unused cache slots: a zero coupling (packed words), or the zero
        // byte past the spins (unit couplings)
        ecache->assign(static_cast<size_t>(n) * p.cache, p.unit ? static_cast<uint32_t>(kResZero) : 0u);
        for (int32_t pos = 0; pos < n; ++pos) {
            const PeriodRec &r = (*recs)[pos];
            for (int32_t u = 0; u < p.cache && r.rp0 + u < r.rp1; ++u) {
                const int32_t e = r.rp0 + u;
                (*ecache)[static_cast<size_t>(pos) * p.cache + u] =
                    p.unit ? static_cast<uint32_t>(col_host[e] + (val_host[e] < 0 ? kResNeg : 0))
                           : static_cast<uint32_t>(col_host[e]) | (static_cast<uint32_t>(val_host[e]) << 16);
            }
        }
    }
    *plan = p;
    return true;
}

hipError_t launch_period(hipStream_t stream, const DevGraph &g, const DevRun &run,
                         const PeriodPlan &plan, const PeriodRec *recs, const PeriodClass *classes,
                         const uint32_t *ecache, int32_t t_begin, int32_t t_end) {
    if (t_end <= t_begin) return hipSuccess;
    if (plan.nclass < 1 || plan.nclass > kPeriodMaxClasses || run.t_res < 1 ||
        (plan.pk32 && !g.pk32) || (plan.resident_k > 0 && (!g.pk32 || !ecache)))
        return hipErrorInvalidValue;
    PeriodArgs a{};
    a.n = g.n;
    a.t4 = run.t4;
    a.t_begin = t_begin;
    a.t_end = t_end;
    a.t_res = run.t_res;
    a.nclass = plan.nclass;
    a.sbuf = plan.sbuf;
    a.nnz = static_cast<int32_t>(g.nnz);
    a.recs = recs;
    a.classes = classes;
    a.pk32 = g.pk32;
    a.col = g.col;
    a.val = g.val;
    a.i0 = run.i0;
    a.k0 = run.key0;
    a.k1 = run.key1;
    a.spins = run.spins;
    const int32_t grid = run.trials;
    if (plan.resident_k > 0) {
        if (static_cast<int64_t>(plan.resident_k) * plan.block < g.n) return hipErrorInvalidValue;
        if (plan.cache != resident_cache(plan.resident_k) ||
            plan.resident_k != resident_k_for(g.n, plan.block))
            return hipErrorInvalidValue;
        switch (plan.block * 16 + plan.resident_k) {
            case 1024 * 16 + 1: return launch_resident_k<1, 16, 1024>(stream, a, plan, ecache, grid);
            case 1024 * 16 + 2: return launch_resident_k<2, 12, 1024>(stream, a, plan, ecache, grid);
            case 512 * 16 + 1: return launch_resident_k<1, 16, 512>(stream, a, plan, ecache, grid);
            case 512 * 16 + 2: return launch_resident_k<2, 12, 512>(stream, a, plan, ecache, grid);
            case 512 * 16 + 4: return launch_resident_k<4, 12, 512>(stream, a, plan, ecache, grid);
            case 256 * 16 + 1: return launch_resident_k<1, 16, 256>(stream, a, plan, ecache, grid);
            case 256 * 16 + 2: return launch_resident_k<2, 12, 256>(stream, a, plan, ecache, grid);
            case 256 * 16 + 4: return launch_resident_k<4, 12, 256>(stream, a, plan, ecache, grid);
            case 256 * 16 + 8: return launch_resident_k<8, 8, 256>(stream, a, plan, ecache, grid);
            default: return hipErrorInvalidValue;
        }
    }
    if (plan.in_lds)
        return plan.pk32 ? launch_block<true, true>(stream, a, plan, grid)
                         : launch_block<true, false>(stream, a, plan, grid);
    return plan.pk32 ? launch_block<false, true>(stream, a, plan, grid)
                     : launch_block<false, false>(stream, a, plan, grid);
}

}  // namespace psa
