// dense.hip -- dense matrix-core path of the local field (gfx950).
//
// For graphs whose rows are long, one synchronous step is a product of the
// dense coupling matrix with the spins of all trials,
//     L[i][k] = h_i + sum_j J_ij m_j,k      (exact integer sums),
// computed on the matrix cores, followed by the p-bit update of Eq. 6 in the
// same kernel.  One launch of dense_step_kernel advances one step of every
// dense run in a work list (run, 256-row group, trial tile), with the step
// loop on the host, because a step needs the whole previous state of its
// run; dense_steps_kernel runs all steps of a quantum in one launch instead,
// each work item waiting on a per-run counter of the previous step.
//
// Coupling encodings (per graph, chosen at build time):
//   kDenseI8  int8 [np][np], row-major, zero padding (any |J| <= 127), with
//             int8 spins, through v_mfma_i32_16x16x64_i8 (np a multiple of
//             128);
//   kDenseT2  2-bit fields f in {0, +1, -1} with J = scale * f, for graphs
//             whose couplings share one magnitude (unit and +-1 weights),
//             with fp4 (e2m1) spins, through v_mfma_f32_16x16x128_f8f6f4 in
//             its fp4 x fp4 form (np a multiple of 256).  0, +1 and -1 are
//             exact fp4 values (codes 0x0, 0x2, 0xA), every product is 0 or
//             +-1 and every partial sum an integer below 2^24 (the field
//             bound), so the f32 sums are the exact integers.  Four times
//             fewer coupling bytes than int8, and twice the depth per matrix
//             instruction at the int8 instruction's issue cost.
//   kDenseB1  1-bit fields f in {0, 1} with J = scale * f, for graphs whose
//             couplings all have one value (+1-weight MAX-CUT, all
//             ferromagnetic): the fp4 path with half the coupling bytes of
//             kDenseT2 (np a multiple of 256).  B1 words: one 32-bit word per
//             lane, row block and 128-column k-step holds the lane's 32
//             columns, column 32 g + 8 d + q in bit 4q + d, so that operand
//             dword d is w shifted by 1 - d and masked with 0x22222222 (fp4
//             1.0 where the bit is set); per 64-row tile and 256-column chunk,
//             2 KB as two 1 KB halves (one per k-step) of [64 lanes][4 row
//             blocks], two 16-byte loads per lane and chunk.
//   T2 words: the fp4 operand of one lane is four dwords d = 0..3 whose
//   nibble q is column 32 g + 8 d + q of the 128-column k-step (g = lane /
//   16); one 32-bit word w holds two of them, dword 2 v in bits 4q + 1 (set:
//   nonzero) and 4q + 3 (set: negative) of w, dword 2 v + 1 in bits 4q and
//   4q + 2 of w, so that the dwords are w & 0xAAAAAAAA and (w << 1) &
//   0xAAAAAAAA: fp4 1.0 = 0b0010, -1.0 = 0b1010.  The words are tiled in the
//   order a wave loads them: per 64-row tile and 256-column chunk, 4 KB as
//   four 1 KB quarters of [64 lanes][4 words]; word j of lane l in quarter Q
//   is row 16 (2 (Q % 2) + j / 2) + l % 16 of the tile, k-step Q / 2 of the
//   chunk, pair j % 2 (dwords 2 (j % 2) and 2 (j % 2) + 1) of lane group
//   l / 16.  A lane's operands for a chunk are four 16-byte loads, and each
//   load instruction of the wave reads 1 KB contiguous.
//
// Spins M per buffer, trial-major with the p-bit index contiguous, tp =
// trials rounded up to the trial tile, two buffers by step parity: int8
// [tp][np] (+1 = 0x01, -1 = 0xFF), or fp4 [tp][np / 2] bytes (p-bit 2b in the
// low nibble of byte b; +1 = 0x2, -1 = 0xA).  Either way one chunk of a
// trial's spins is 128 bytes: 128 int8 or 256 fp4 columns.
//
// MFMA operand layout: lane l supplies A[row l%16][16 bytes of k at group l/16]
// and B[the same k][col l%16]; for the 16x16x64 int8 form those are 16 int8,
// for the fp4 form 32 nibbles.  Lane l receives D[row (l/16)*4 + r][col l%16]
// in its four accumulators r = 0..3.  The four rows of a lane are four
// consecutive p-bits 4m..4m+3 of one trial: exactly the p-bits one Philox
// block serves, so the epilogue draws one r block (and one gate block) per
// lane, row block and trial column.
//
// Workgroup: 4 waves x 64 rows (four 16-row blocks per wave) against one trial
// tile of 16 NB trials.  The trial tile's spins stream through LDS in chunks
// of 128 bytes per trial (double-buffered, one barrier per chunk); each wave
// reads its own coupling rows straight from memory, one chunk ahead of the
// matrix work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kChunkBytes = 128;               // bytes of one trial's spins per LDS chunk
constexpr int kLdsStride = kChunkBytes + 16;   // padded LDS row of the spin tile (bytes)
constexpr int kWaveRows = 64;                  // four 16-row blocks per wave
constexpr int kGroupRows = 256;                // rows per workgroup

// Per encoding: columns per chunk, spin bits, spin codes, accumulator type.
template <int ENC>
struct Enc;
template <>
struct Enc<kDenseI8> {
    static constexpr int kCols = 128;
    static constexpr int kBits = 8;
    static constexpr uint32_t kUp = 0x01u, kDown = 0xFFu;
    using Acc = v4i;
};
template <>
struct Enc<kDenseT2> {
    static constexpr int kCols = 256;
    static constexpr int kBits = 4;
    static constexpr uint32_t kUp = 0x2u, kDown = 0xAu;
    using Acc = v4f;
};
template <>
struct Enc<kDenseB1> : Enc<kDenseT2> {};

// One pair word of 2-bit fields -> two fp4 dwords (see the T2 layout).
constexpr uint32_t kF4Mask = 0xAAAAAAAAu;
__device__ __forceinline__ v8i f4_operand(uint32_t w0, uint32_t w1) {
    return v8i{static_cast<int>(w0 & kF4Mask), static_cast<int>((w0 << 1) & kF4Mask),
               static_cast<int>(w1 & kF4Mask), static_cast<int>((w1 << 1) & kF4Mask), 0, 0, 0, 0};
}
__device__ __forceinline__ v8i f4_widen(const v4i b) { return v8i{b.x, b.y, b.z, b.w, 0, 0, 0, 0}; }
// One word of 1-bit fields -> the four fp4 dwords (see the B1 layout).
constexpr uint32_t kB1Mask = 0x22222222u;
__device__ __forceinline__ v8i b1_operand(uint32_t w) {
    return v8i{static_cast<int>((w << 1) & kB1Mask), static_cast<int>(w & kB1Mask),
               static_cast<int>((w >> 1) & kB1Mask), static_cast<int>((w >> 2) & kB1Mask), 0, 0, 0, 0};
}

// Device-global views of pointers read from the job table (so that loads
// are global, not flat, and do not wait on LDS traffic).
template <typename T>
using gptr = const T __attribute__((address_space(1))) *;
template <typename T, typename P>
__device__ __forceinline__ gptr<T> as_global(P p) {
    return (gptr<T>)(p);
}

template <int ENC>
struct AFrag;
template <>
struct AFrag<kDenseI8> {
    v4i v[2][4];  // k-tile, row block
};
template <>
struct AFrag<kDenseT2> {
    v4i q[4];  // quarter Q, word j: row block 2 (Q % 2) + j / 2, k-step Q / 2, pair j % 2
};
template <>
struct AFrag<kDenseB1> {
    v4i h[2];  // half H = k-step, word j = row block
};

// NB = 16-trial blocks per workgroup (trial tile = 16 NB).  MODE: what every
// run of the launch is -- kDenseAny: tested at run time; kDensePlain: pSA with
// one sub-step per step (no held inputs, windows or periods), so the epilogue
// carries no run-time mode tests; kDenseIdentity: that, and every p-bit has
// lambda = 1, delta = 0 and no timing gate, so the pre-activation is the one
// product I0 (float)L (exactly the general (I0 lambda)((float)L + delta) at
// those values) and no gate word is drawn.
enum : int { kDenseAny = 0, kDensePlain = 1, kDenseIdentity = 2 };
// Spin-buffer accesses of a step that other workgroups' steps read: with
// COH, buffer loads and stores at device (agent) coherence -- they bypass the
// per-XCD L2 copies of the lines -- so that the persistent launch needs no
// cache write-back or invalidation between dependent steps.
constexpr int kCohAux = 16;                  // cache policy bits: device scope
constexpr int kRsrcWord3 = 0x00020000;       // raw buffer resource, gfx9 family

// One work item of one step: w = (job, row group, trial tile, -), job < 0 an
// empty slot; bt the workgroup's two LDS spin chunks.  Every thread of the
// workgroup calls it (it holds workgroup barriers).
template <int NB, int ENC, int MODE, bool COH>
__device__ __forceinline__ void dense_task(const DenseJob *__restrict__ jobs, const int4 w, int32_t t_off,
                                           int8_t (*__restrict__ bt)[16 * NB * kLdsStride]) {
    using E = Enc<ENC>;
    using Acc = typename E::Acc;
    constexpr bool kFp4 = ENC != kDenseI8;
    constexpr bool PLAIN = MODE != kDenseAny;
    constexpr int kTrials = 16 * NB;
    constexpr int kBVec = kTrials * (kChunkBytes / 16);  // 16-byte pieces of one spin chunk
    constexpr int kBPer = (kBVec + 255) / 256;  // 1 or 2
    if (w.x < 0) return;
    const DenseJob &jb = jobs[w.x];
    // launch t_off advances sub-step t_off of this run's sequence: one
    // sub-step per step, or t_res of them in period mode; tau counts
    // sub-steps from the start of the anneal, t is the step (cycle) of tau
    const bool period_mode = !PLAIN && jb.t_res > 0;
    const int32_t u = period_mode ? jb.t_res : 1;
    if (t_off >= (jb.t_end - jb.t) * u) return;
    const uint32_t tau = static_cast<uint32_t>(jb.t * u + t_off);
    const int32_t t = PLAIN ? static_cast<int32_t>(tau) : static_cast<int32_t>(tau / static_cast<uint32_t>(u));
    const int32_t np = jb.np;
    const int32_t rowb = np * E::kBits / 8;  // bytes per trial row of a spin buffer
    const int32_t trial0 = w.z * kTrials;
    const int8_t *__restrict__ cur = (t_off & 1) ? jb.m1 : jb.m0;
    int8_t *__restrict__ nxt = (t_off & 1) ? jb.m0 : jb.m1;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15;
    const int kgrp = (lane >> 4) * 16;
    const int32_t wrow0 = w.y * kGroupRows + wave * kWaveRows;
    // np is a multiple of 128: a wave's 64 rows are all in or all out.  A
    // wave past the end multiplies the last 64 rows again (no branches in the
    // main loop) and skips the epilogue.
    const bool active = wrow0 < np;
    const int32_t arow0 = active ? wrow0 : np - kWaveRows;

    static_assert(kBVec == 128 || kBVec % 256 == 0, "spin chunk split");
    // spin chunk kc+1 staged in registers while chunk kc is multiplied; with
    // a 128-piece chunk the upper half of the threads repeat the lower half
    // (same bytes to the same LDS place), keeping the loop free of branches
    v4i breg0, breg1;
    const int c0 = static_cast<int>(threadIdx.x) % kBVec;
    const gptr<int8_t> gcur = as_global<int8_t>(cur);
    const int32_t buf_bytes = jb.tp * rowb;
    const __amdgpu_buffer_rsrc_t rcur =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t *>(cur), 0, buf_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rnxt = __builtin_amdgcn_make_buffer_rsrc(nxt, 0, buf_bytes, kRsrcWord3);
    auto load16 = [&](int32_t off) -> v4i {
        if constexpr (COH)
            return __builtin_amdgcn_raw_buffer_load_b128(rcur, off, 0, kCohAux);
        else
            return *as_global<v4i>(gcur + off);
    };
    auto fetch_b = [&](int kc) {
        breg0 = load16((trial0 + (c0 >> 3)) * rowb + kc * kChunkBytes + (c0 & 7) * 16);
        if constexpr (kBPer == 2) {
            const int c = c0 + 256;
            breg1 = load16((trial0 + (c >> 3)) * rowb + kc * kChunkBytes + (c & 7) * 16);
        }
    };
    auto store_b = [&](int buf) {
        *reinterpret_cast<v4i *>(&bt[buf][(c0 >> 3) * kLdsStride + (c0 & 7) * 16]) = breg0;
        if constexpr (kBPer == 2) {
            const int c = c0 + 256;
            *reinterpret_cast<v4i *>(&bt[buf][(c >> 3) * kLdsStride + (c & 7) * 16]) = breg1;
        }
    };
    const int nkc = np / E::kCols;
    auto fetch_a = [&](int kc, AFrag<ENC> &dst) {
        if constexpr (ENC == kDenseI8) {
            const gptr<int8_t> J = as_global<int8_t>(jb.J);
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const size_t row = static_cast<size_t>(arow0 + rb * 16 + lr);
                    dst.v[kt][rb] = *as_global<v4i>(J + row * np + kc * E::kCols + kt * 64 + kgrp);
                }
        } else if constexpr (ENC == kDenseT2) {
            const gptr<v4i> J = as_global<v4i>(jb.J);
            const size_t tile = (static_cast<size_t>(arow0 / kWaveRows) * nkc + kc) * 4;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) dst.q[qq] = J[(tile + qq) * 64 + lane];
        } else {
            const gptr<v4i> J = as_global<v4i>(jb.J);
            const size_t tile = (static_cast<size_t>(arow0 / kWaveRows) * nkc + kc) * 2;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) dst.h[hh] = J[(tile + hh) * 64 + lane];
        }
    };

    Acc acc[4][NB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = Acc{0, 0, 0, 0};

    // one chunk: two k-steps of 64 int8 or 128 fp4 columns (64 bytes of each
    // trial's spins each)
    auto compute = [&](int buf, const AFrag<ENC> &af) {
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            v4i b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                b[nb] = *reinterpret_cast<const v4i *>(&bt[buf][(nb * 16 + lr) * kLdsStride + kt * 64 + kgrp]);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                if constexpr (ENC == kDenseI8) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[rb][nb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af.v[kt][rb], b[nb], acc[rb][nb], 0, 0, 0);
                } else {
                    v8i a;
                    if constexpr (ENC == kDenseT2) {
                        const v4i &qw = af.q[kt * 2 + (rb >> 1)];
                        a = f4_operand(static_cast<uint32_t>(qw[(rb & 1) * 2]),
                                       static_cast<uint32_t>(qw[(rb & 1) * 2 + 1]));
                    } else {
                        a = b1_operand(static_cast<uint32_t>(af.h[kt][rb]));
                    }
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[rb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            a, f4_widen(b[nb]), acc[rb][nb], 4, 4, 0, 0, 0, 0);  // fp4 x fp4, no scaling
                }
            }
        }
    };
    // one chunk: prefetch chunk kc+1 (the last chunk fetches itself again)
    // -- spins into registers, couplings into `pre` --, multiply chunk kc,
    // then publish the prefetched spins into the other LDS buffer
    auto chunk = [&](int kc, const AFrag<ENC> &use, AFrag<ENC> &pre) {
        const int kn = kc + 1 < nkc ? kc + 1 : kc;
        fetch_b(kn);
        fetch_a(kn, pre);
        // keep the prefetch ahead of the matrix work (the scheduler would
        // otherwise sink the loads next to their first use)
        __builtin_amdgcn_sched_barrier(0);
        compute(kc & 1, use);
        __builtin_amdgcn_sched_barrier(0);
        store_b((kc + 1) & 1);
        __syncthreads();
    };

    AFrag<ENC> fa, fb;
    fetch_b(0);
    store_b(0);
    fetch_a(0, fa);
    __syncthreads();
    for (int kc = 0; kc < nkc; kc += 2) {
        chunk(kc, fa, fb);
        if (kc + 1 < nkc) chunk(kc + 1, fb, fa);
    }
    if (!active) return;

    // epilogue: lane owns p-bits 4m..4m+3 of each row block for trial columns
    // nb.  The sum of a p-bit is exact in either accumulator type, and so is
    // its conversion: L = h + scale * sum as an integer, or (float)L by one
    // fma (scale * sum and the total are integers below 2^24).
    const float i0t = jb.i0[t];
    // the spins of p-bits i0..i0+3 of trial k in a buffer, 32 or 16 bits
    auto spin_off = [&](uint32_t k, int32_t i0) {
        return static_cast<int32_t>(k) * rowb + (i0 * E::kBits >> 3);
    };
    auto store4 = [&](uint32_t k, int32_t i0, uint32_t out) {
        const int32_t off = spin_off(k, i0);
        if constexpr (COH && kFp4)
            __builtin_amdgcn_raw_buffer_store_b16(static_cast<uint16_t>(out), rnxt, off, 0, kCohAux);
        else if constexpr (COH)
            __builtin_amdgcn_raw_buffer_store_b32(out, rnxt, off, 0, kCohAux);
        else if constexpr (kFp4)
            *reinterpret_cast<uint16_t *>(nxt + off) = static_cast<uint16_t>(out);
        else
            *reinterpret_cast<uint32_t *>(nxt + off) = out;
    };
    auto load4 = [&](uint32_t k, int32_t i0) -> uint32_t {
        const int32_t off = spin_off(k, i0);
        if constexpr (COH && kFp4)
            return __builtin_amdgcn_raw_buffer_load_b16(rcur, off, 0, kCohAux);
        else if constexpr (COH)
            return __builtin_amdgcn_raw_buffer_load_b32(rcur, off, 0, kCohAux);
        else if constexpr (kFp4)
            return *reinterpret_cast<const uint16_t *>(cur + off);
        else
            return *reinterpret_cast<const uint32_t *>(cur + off);
    };
    if constexpr (MODE == kDenseIdentity) {
        // one r block and four products per (row block, trial block) pair; the
        // pairs unrolled with constant accumulator indices, two per scheduling
        // region (their chains are independent), the key schedule formed once.
        // Each decision is taken from the tanh estimate, its spin code from
        // the sign of the estimate's distance to r; when some lane of the wave
        // holds an estimate within 2^-16 of r (about one pair in 250), the
        // pair's codes are taken from the exact recipe instead -- one uniform
        // branch per pair, none per p-bit.  Padding p-bits and trials are
        // written too (their rows and columns of J are zero, and the read-out
        // skips them).
        const int32_t scale = jb.scale;
        const float scalef = static_cast<float>(scale);
        const uint32_t kpos = static_cast<uint32_t>(trial0 + lr);
        const PhiloxKeys keys = philox_keys(jb.k0, jb.k1);
        const gptr<v4i> hvec = as_global<v4i>(jb.h);
        // codes of four up spins, and the bits that turn a code into down
        constexpr uint32_t kUp4 = kFp4 ? 0x2222u : 0x01010101u;
        constexpr uint32_t kFlip = kFp4 ? 0x8u : 0xFEu;
#pragma unroll
        for (int e = 0; e < 4 * NB; ++e) {
            const int rb = e / NB, nb = e % NB;
            const int32_t i0 = wrow0 + rb * 16 + (lane >> 4) * 4;
            const uint32_t k = kpos + static_cast<uint32_t>(nb * 16);
            const v4i hh = hvec[(i0 < jb.n4 ? i0 : 0) >> 2];
            const Words4 r = philox4x32_10(tau, static_cast<uint32_t>(i0 >> 2), k, kTagR, keys);
            const int32_t hv[4] = {hh[0], hh[1], hh[2], hh[3]};
            const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
            float x[4];
            uint32_t out = kUp4;
            bool close = false;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                float Lf;
                if constexpr (kFp4)
                    Lf = fmaf(scalef, acc[rb][nb][p], static_cast<float>(hv[p]));
                else
                    Lf = static_cast<float>(hv[p] + scale * acc[rb][nb][p]);
                x[p] = i0t * Lf;
                const float diff = tanh_estimate_minus(x[p], r_of(rw[p]));
                close = close || !estimate_decides(diff);
                // diff < 0 (sign bit set): down
                const uint32_t neg = static_cast<uint32_t>(static_cast<int32_t>(__float_as_uint(diff)) >> 31);
                out ^= (neg & kFlip) << (E::kBits * p);
            }
            if (__ballot(close) != 0u) {
                out = 0u;
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    out |= (tanh_f32(x[p]) > r_of(rw[p]) ? E::kUp : E::kDown) << (E::kBits * p);
            }
            store4(k, i0, out);
            if (e & 1) __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    // the other modes: the (row block, trial block) pairs run as a loop with a
    // uniform index, so the body -- Philox blocks and four activations -- is
    // emitted once per pass, keeping few registers live.
    const int32_t scale = jb.scale;
    const InputState st{jb.xs, jb.stall24, jb.ring, jb.alpha, jb.n4};
    auto update = [&](int e, const Acc a4) __attribute__((always_inline)) {
        const int rb = e / NB, nb = e % NB;
        const int32_t i0 = wrow0 + rb * 16 + (lane >> 4) * 4;
        const int32_t k = trial0 + nb * 16 + lr;
        // lanes past the padded p-bits or trials compute on clamped inputs
        // and store nothing (straight-line code, so that two passes interleave)
        const bool valid = i0 < jb.n4 && k < jb.t4;
        const int32_t ic = valid ? i0 : 0;
        const int32_t m = i0 >> 2;
        const int4 hh = *reinterpret_cast<const int4 *>(jb.h + ic);
        const uint4 th = *reinterpret_cast<const uint4 *>(jb.thr + ic);
        const float4 lm = *reinterpret_cast<const float4 *>(jb.lam + ic);
        const float4 dl = *reinterpret_cast<const float4 *>(jb.dlt + ic);
        const InputState sv{valid ? st.xs : nullptr, st.s24, valid ? st.ring : nullptr, st.alpha, st.n4};
        const int32_t hv[4] = {hh.x, hh.y, hh.z, hh.w};
        const uint32_t tv[4] = {th.x, th.y, th.z, th.w};
        const float av[4] = {i0t * lm.x, i0t * lm.y, i0t * lm.z, i0t * lm.w};
        const float dv[4] = {dl.x, dl.y, dl.z, dl.w};
        const bool need_gate = !period_mode && ((tv[0] < kGateOne) | (tv[1] < kGateOne) |
                                                (tv[2] < kGateOne) | (tv[3] < kGateOne));
        uint32_t old = 0u;
        uint32_t gw[4] = {0u, 0u, 0u, 0u};
        if (need_gate || period_mode)  // p-bits that do not fire keep these
            old = load4(static_cast<uint32_t>(k), i0);
        if (need_gate) {
            const Words4 g = philox4x32_10(tau, static_cast<uint32_t>(m),
                                           static_cast<uint32_t>(k), kTagGate, jb.k0, jb.k1);
            gw[0] = g.x;
            gw[1] = g.y;
            gw[2] = g.z;
            gw[3] = g.w;
        }
        const Words4 r = philox4x32_10(tau, static_cast<uint32_t>(m),
                                       static_cast<uint32_t>(k), kTagR, jb.k0, jb.k1);
        const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
        uint32_t sw[4] = {0u, 0u, 0u, 0u};
        if (!PLAIN && sv.xs != nullptr && t > 0) {
            const Words4 b = philox4x32_10(static_cast<uint32_t>(t), static_cast<uint32_t>(m),
                                           static_cast<uint32_t>(k), kTagStall, jb.k0, jb.k1);
            sw[0] = b.x;
            sw[1] = b.y;
            sw[2] = b.z;
            sw[3] = b.w;
        }
        constexpr uint32_t kMask = (1u << E::kBits) - 1u;
        uint32_t out = 0u;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int32_t L = hv[p] + scale * static_cast<int32_t>(a4[p]);
            const float x = PLAIN ? input_of<kAlgPsa>(av[p], dv[p], L, sv, i0 + p, static_cast<uint32_t>(k),
                                                      static_cast<uint32_t>(t), sw[p])
                                  : input_any(av[p], dv[p], L, sv, i0 + p, static_cast<uint32_t>(k),
                                      static_cast<uint32_t>(t), sw[p]);
            const bool up = pbit_up(x, rw[p]);
            const bool fire = period_mode ? period_fires(tau, tv[p])
                                          : (tv[p] >= kGateOne || fires(gw[p], tv[p]));
            const uint32_t ob = (old >> (E::kBits * p)) & kMask;
            out |= (fire ? (up ? E::kUp : E::kDown) : ob) << (E::kBits * p);
        }
        if (valid) store4(static_cast<uint32_t>(k), i0, out);
    };
    // The accumulators move through a queue read only at its head (constant
    // register indices; a loop index into the array would force it into
    // scratch memory).  Two (row block, trial block) pairs per pass: their
    // Philox chains are independent, which doubles the instruction-level
    // parallelism.
    Acc q[4 * NB];
#pragma unroll
    for (int e = 0; e < 4 * NB; ++e) q[e] = acc[e / NB][e % NB];
#pragma unroll 1
    for (int e = 0; e < 4 * NB; e += 2) {
        update(e, q[0]);
        update(e + 1, q[1]);
#pragma unroll
        for (int j = 0; j + 2 < 4 * NB; ++j) q[j] = q[j + 2];
    }
}

template <int NB, int ENC, int MODE>
__global__ __launch_bounds__(256, ENC != kDenseI8 ? 3 : 2) void dense_step_kernel(const DenseJob *__restrict__ jobs,
                                                         const int4 *__restrict__ work, int32_t t_off) {
    __shared__ __align__(16) int8_t bt[2][16 * NB * kLdsStride];
    dense_task<NB, ENC, MODE, false>(jobs, work[blockIdx.x], t_off, bt);
}

// All `steps` steps of a work list in one launch.  The work list is split
// into kDenseQueues queues, each holding whole runs; queue x's task q = s n_x
// + i is its item i of step s.  A workgroup takes tasks in that order from
// its home queue's ticket counter (home: blockIdx mod 8, the XCD it is
// dispatched to, so a run's spin tiles stay in one L2), then from the other
// queues in turn; a task of step s > 0 first waits until every item of its
// run has finished step s - 1 (its run's counter reaches s items).  A task
// only waits on tasks of its own queue with smaller tickets, which running
// workgroups hold, so the waits end whatever number of workgroups the device
// keeps resident; runs, and a run's consecutive steps, overlap (one's
// epilogue with another's matrix loop).  The workgroups of a run may still
// sit on different XCDs, each with its own L2: spins are stored and read at
// device coherence (dense_task's COH accesses, which bypass the L2 copies),
// and a task's stores have completed before its counter increment; no cache
// is written back or invalidated (that would also cost kernels running
// beside it their cached lines).  Runs must be plain pSA (MODE kDensePlain
// or kDenseIdentity: no held inputs or windows, which other tasks would read).
//   sync (words, each counter on its own 128-byte line): queue x's ticket
//   counter at 32 x, the error flag at 32 kDenseQueues, run j's tasks done at
//   32 (kDenseQueues + 1 + j); zero before the launch.  Each wait polls at most
//   max_polls times; past that, or once another workgroup has set the error
//   flag, the workgroup sets the flag and leaves (the host reports it).
template <int NB, int ENC, int MODE>
__global__ __launch_bounds__(256, ENC != kDenseI8 ? 3 : 2) void dense_steps_kernel(
    const DenseJob *__restrict__ jobs, const int4 *__restrict__ work, DenseQueues queues, int32_t steps,
    uint32_t *__restrict__ sync, uint32_t max_polls) {
    __shared__ __align__(16) int8_t bt[2][16 * NB * kLdsStride];
    __shared__ uint32_t s_ticket, s_fail;
    uint32_t *const err = sync + 32 * kDenseQueues;
    uint32_t *const done0 = sync + 32 * (kDenseQueues + 1);
    const int home = static_cast<int>(blockIdx.x % kDenseQueues);
    // Control flow below depends only on wavefront-uniform values (read from
    // LDS with readfirstlane), and the one thread-0 region of an iteration
    // sits between barriers: a loop exit the compiler must treat as divergent
    // lets it split a wavefront's lanes across the loop latch, and that
    // wavefront then meets a different number of barriers than the others.
    int32_t owed = -1;  // run whose counter this workgroup's last task has not yet advanced
    for (int a = 0; a < kDenseQueues; ++a) {
        const int x = (home + a) % kDenseQueues;
        const int32_t items = queues.off[x + 1] - queues.off[x];
        const uint32_t total = static_cast<uint32_t>(steps) * static_cast<uint32_t>(items);
        if (total == 0u) continue;
        for (;;) {
            // the previous task's stores completed in every wavefront (the
            // barrier closing it): publish it, then take the next ticket
            if (threadIdx.x == 0) {
                if (owed >= 0)
                    __hip_atomic_fetch_add(done0 + 32 * owed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_fail = f;
                s_ticket = f ? total
                             : __hip_atomic_fetch_add(sync + 32 * x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            owed = -1;
            __syncthreads();
            const uint32_t ticket = __builtin_amdgcn_readfirstlane(s_ticket);
            const uint32_t failed = __builtin_amdgcn_readfirstlane(s_fail);
            __syncthreads();  // read before thread 0 writes them again
            if (failed) return;
            if (ticket >= total) break;  // queue drained: the next one
            const int32_t s = static_cast<int32_t>(ticket / static_cast<uint32_t>(items));
            const int4 w = work[queues.off[x] + static_cast<int32_t>(ticket % static_cast<uint32_t>(items))];
            if (s > 0) {
                if (threadIdx.x == 0) {
                    const uint32_t need = static_cast<uint32_t>(s) * static_cast<uint32_t>(jobs[w.x].items);
                    const uint32_t *done = done0 + 32 * w.x;
                    uint32_t fail = 1u;
                    for (uint32_t n = 0; n < max_polls; ++n) {
                        if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
                            fail = 0u;
                            break;
                        }
                        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                        __builtin_amdgcn_s_sleep(4);
                    }
                    if (fail) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_fail = fail;
                }
                __syncthreads();
                const uint32_t waited_out = __builtin_amdgcn_readfirstlane(s_fail);
                if (waited_out) return;
            }
            dense_task<NB, ENC, MODE, true>(jobs, w, s, bt);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's spin stores complete
            __syncthreads();
            owed = w.x;
        }
    }
    if (threadIdx.x == 0 && owed >= 0)
        __hip_atomic_fetch_add(done0 + 32 * owed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void zero_words_kernel(uint32_t *__restrict__ p, int32_t count) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < count) p[i] = 0u;
}

// [n][t4] (trials innermost) <-> [tp][np] (p-bits contiguous, int8), or
// [tp][np / 2] bytes of fp4 nibbles; padding p-bits and trials of the dense
// layout are +1.
__global__ void to_dense_kernel(int32_t n, int32_t t4, int32_t np, int32_t tp,
                                const int8_t *__restrict__ spins, int8_t *__restrict__ m) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(tp) * np) return;
    const int32_t k = static_cast<int32_t>(idx / np);
    const int32_t i = static_cast<int32_t>(idx % np);
    m[idx] = (i < n && k < t4) ? spins[static_cast<size_t>(i) * t4 + k] : int8_t(1);
}

__global__ void to_dense_f4_kernel(int32_t n, int32_t t4, int32_t np, int32_t tp,
                                   const int8_t *__restrict__ spins, uint8_t *__restrict__ m) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int32_t half = np / 2;
    if (idx >= static_cast<int64_t>(tp) * half) return;
    const int32_t k = static_cast<int32_t>(idx / half);
    const int32_t i = 2 * static_cast<int32_t>(idx % half);
    auto code = [&](int32_t p) -> uint32_t {
        return (p < n && k < t4 && spins[static_cast<size_t>(p) * t4 + k] < 0) ? 0xAu : 0x2u;
    };
    m[idx] = static_cast<uint8_t>(code(i) | code(i + 1) << 4);
}

__global__ void from_dense_kernel(int32_t n, int32_t t4, int32_t np, const int8_t *__restrict__ m,
                                  int8_t *__restrict__ spins) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * t4) return;
    const int32_t i = static_cast<int32_t>(idx / t4);
    const int32_t k = static_cast<int32_t>(idx % t4);
    spins[idx] = m[static_cast<size_t>(k) * np + i];
}

__global__ void from_dense_f4_kernel(int32_t n, int32_t t4, int32_t np, const uint8_t *__restrict__ m,
                                     int8_t *__restrict__ spins) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * t4) return;
    const int32_t i = static_cast<int32_t>(idx / t4);
    const int32_t k = static_cast<int32_t>(idx % t4);
    const uint32_t nib = (m[static_cast<size_t>(k) * (np / 2) + i / 2] >> (4 * (i & 1))) & 0xFu;
    spins[idx] = nib == 0x2u ? int8_t(1) : int8_t(-1);
}

template <int ENC, int MODE>
hipError_t launch_dense_enc(hipStream_t stream, const DenseJob *jobs, const int4 *work, int32_t nwork,
                            int32_t nb, int32_t s) {
    switch (nb) {
        case 1: hipLaunchKernelGGL((dense_step_kernel<1, ENC, MODE>), dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
        case 2: hipLaunchKernelGGL((dense_step_kernel<2, ENC, MODE>), dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
        case 4: hipLaunchKernelGGL((dense_step_kernel<4, ENC, MODE>), dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ENC>
hipError_t launch_dense_mode(hipStream_t stream, const DenseJob *jobs, const int4 *work, int32_t nwork,
                             int32_t nb, int32_t mode, int32_t s) {
    switch (mode) {
        case kDenseAny: return launch_dense_enc<ENC, kDenseAny>(stream, jobs, work, nwork, nb, s);
        case kDensePlain: return launch_dense_enc<ENC, kDensePlain>(stream, jobs, work, nwork, nb, s);
        case kDenseIdentity: return launch_dense_enc<ENC, kDenseIdentity>(stream, jobs, work, nwork, nb, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_dense_steps(hipStream_t stream, const DenseJob *jobs, const int4 *work,
                              int32_t nwork, int32_t nb, int32_t enc, int32_t mode, int32_t steps) {
    if (nwork <= 0) return hipSuccess;
    for (int32_t s = 0; s < steps; ++s) {
        const hipError_t e = enc == kDenseB1   ? launch_dense_mode<kDenseB1>(stream, jobs, work, nwork, nb, mode, s)
                             : enc == kDenseT2 ? launch_dense_mode<kDenseT2>(stream, jobs, work, nwork, nb, mode, s)
                                               : launch_dense_mode<kDenseI8>(stream, jobs, work, nwork, nb, mode, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int ENC, int MODE>
hipError_t launch_persistent_enc(hipStream_t stream, const DenseJob *jobs, const int4 *work, const DenseQueues &q,
                                 int32_t nb, int32_t steps, uint32_t *sync, uint32_t max_polls, int32_t num_cu) {
    void (*fn)(const DenseJob *, const int4 *, DenseQueues, int32_t, uint32_t *, uint32_t);
    switch (nb) {
        case 1: fn = dense_steps_kernel<1, ENC, MODE>; break;
        case 2: fn = dense_steps_kernel<2, ENC, MODE>; break;
        case 4: fn = dense_steps_kernel<4, ENC, MODE>; break;
        default: return hipErrorInvalidValue;
    }
    int per_cu = 0;
    const hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
    if (oe != hipSuccess) return oe;
    const int64_t tasks = static_cast<int64_t>(steps) * q.off[kDenseQueues];
    const int64_t slots = static_cast<int64_t>(std::max(per_cu, 1)) * std::max(num_cu, 1);
    const int64_t grid = std::max<int64_t>(1, std::min(tasks, slots));
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, jobs, work, q, steps, sync,
                       max_polls);
    return hipGetLastError();
}

int32_t dense_sync_words(int32_t jobs) { return 32 * (kDenseQueues + 1 + jobs); }

hipError_t launch_dense_persistent(hipStream_t stream, const DenseJob *jobs, const int4 *work,
                                   const DenseQueues &q, int32_t nb, int32_t enc, int32_t mode, int32_t steps,
                                   uint32_t *sync, int32_t sync_words, uint32_t max_polls, int32_t num_cu) {
    if (q.off[kDenseQueues] <= 0 || steps <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3(static_cast<unsigned>((sync_words + 255) / 256)), dim3(256), 0,
                       stream, sync, sync_words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto go = [&](auto enc_tag) -> hipError_t {
        constexpr int ENC = decltype(enc_tag)::value;
        switch (mode) {
            case kDensePlain: return launch_persistent_enc<ENC, kDensePlain>(stream, jobs, work, q, nb, steps, sync, max_polls, num_cu);
            case kDenseIdentity: return launch_persistent_enc<ENC, kDenseIdentity>(stream, jobs, work, q, nb, steps, sync, max_polls, num_cu);
            default: return hipErrorInvalidValue;
        }
    };
    return enc == kDenseB1   ? go(std::integral_constant<int, kDenseB1>{})
           : enc == kDenseT2 ? go(std::integral_constant<int, kDenseT2>{})
                             : go(std::integral_constant<int, kDenseI8>{});
}

hipError_t launch_to_dense(hipStream_t stream, int32_t enc, int32_t n, int32_t t4, int32_t np, int32_t tp,
                           const int8_t *spins, int8_t *m) {
    const int64_t items = static_cast<int64_t>(tp) * (dense_fp4(enc) ? np / 2 : np);
    const dim3 grid(static_cast<unsigned>((items + 255) / 256));
    if (dense_fp4(enc))
        hipLaunchKernelGGL(to_dense_f4_kernel, grid, dim3(256), 0, stream, n, t4, np, tp, spins,
                           reinterpret_cast<uint8_t *>(m));
    else
        hipLaunchKernelGGL(to_dense_kernel, grid, dim3(256), 0, stream, n, t4, np, tp, spins, m);
    return hipGetLastError();
}

hipError_t launch_from_dense(hipStream_t stream, int32_t enc, int32_t n, int32_t t4, int32_t np,
                             const int8_t *m, int8_t *spins) {
    const int64_t items = static_cast<int64_t>(n) * t4;
    const dim3 grid(static_cast<unsigned>((items + 255) / 256));
    if (dense_fp4(enc))
        hipLaunchKernelGGL(from_dense_f4_kernel, grid, dim3(256), 0, stream, n, t4, np,
                           reinterpret_cast<const uint8_t *>(m), spins);
    else
        hipLaunchKernelGGL(from_dense_kernel, grid, dim3(256), 0, stream, n, t4, np, m, spins);
    return hipGetLastError();
}

}  // namespace psa
