// dense.hip -- dense matrix-core path of the local field (gfx950).
//
// For graphs whose rows are long, one synchronous step is a product of the
// dense coupling matrix with the spins of all trials,
//     L[i][k] = h_i + sum_j J_ij m_j,k      (int8 x int8 -> int32, exact),
// computed with v_mfma_i32_16x16x64_i8, followed by the p-bit update of
// Eq. 6 in the same kernel.  One launch advances one step of every dense run
// in a work list (run, 256-row group, trial tile); the step loop is on the
// host, because a step needs the whole previous state of its run.
//
// Coupling encodings (per graph, chosen at build time):
//   kDenseI8  int8 [np][np], row-major, zero padding (any |J| <= 127);
//   kDenseT2  2-bit fields f in {0, +1, -1} with J = scale * f, for graphs
//             whose couplings share one magnitude (unit and +-1 weights).
//             Four times fewer bytes than int8; unpacked to int8 in
//             registers with v_perm_b32 just before the matrix instruction.
//   T2 words: one uint32 per (row i, 64-column k-tile, 16-column lane group
//   g); column 64 ktile + 16 g + 4d + b sits in bits 8b + 2d .. 8b + 2d + 1
//   (d = dword of the operand, b = byte): fields of even dwords in bits 0-1
//   of a byte (of word >> 4 for d = 2), of odd dwords in bits 2-3.  The
//   words are tiled in the order a wave loads them: per 64-row tile and
//   128-column chunk, 2 KB as two 1 KB halves of [64 lanes][4 words]; word
//   j of lane l in half h is row
//   16 (2h + j/2) + l % 16 of the tile, k-tile j % 2 of the chunk, group
//   l / 16.  A lane's fragments for a chunk are two 16-byte loads, and each
//   load instruction of the wave reads 1 KB contiguous.
//
// Spins M: int8 [tp][np] per buffer (trial-major, p-bit index contiguous), tp
// = trials rounded up to the trial tile; two buffers by step parity.
//
// MFMA operand layout (16x16x64, int8): lane l supplies A[row l%16][k (l/16)*16
// .. +15] and B[k (l/16)*16 .. +15][col l%16] as 16 bytes each, and receives
// D[row (l/16)*4 + r][col l%16] in its four accumulators r = 0..3.  The four
// rows of a lane are four consecutive p-bits 4m..4m+3 of one trial: exactly
// the p-bits one Philox block serves, so the epilogue draws one r block (and
// one gate block) per lane, row block and trial column.
//
// Workgroup: 4 waves x 64 rows (four 16-row blocks per wave) against one trial
// tile of 16 NB trials.  The trial tile's spins stream through LDS in chunks
// of 128 columns (double-buffered, one barrier per chunk); each wave reads its
// own coupling rows straight from memory, one chunk ahead of the matrix work.
#include <hip/hip_runtime.h>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kKC = 128;             // columns per LDS chunk (two k-tiles)
constexpr int kLdsStride = kKC + 16; // padded LDS row of the spin tile (bytes)
constexpr int kWaveRows = 64;        // four 16-row blocks per wave
constexpr int kGroupRows = 256;      // rows per workgroup

// Field f in {0, 1, 2} -> byte {0x00, 0x01, 0xFF}, four bytes at once.
// Even dwords: the field in bits 0-1 of each byte is a selector of the low
// source's bytes 0x00, 0x01, 0xFF.  Odd dwords: the field in bits 2-3, masked
// in place, is the selector 0, 4 or 8: the low source's byte 0 (0x00), the
// high source's byte 0 (0x01), or the sign of the low source's byte 1 (0xFF).
// So one mask per dword and one shift per pair, no shift per dword.
__device__ __forceinline__ int32_t t2_even(uint32_t w) {
    return static_cast<int32_t>(__builtin_amdgcn_perm(0u, 0x00FF0100u, w & 0x03030303u));
}
__device__ __forceinline__ int32_t t2_odd(uint32_t w) {
    return static_cast<int32_t>(__builtin_amdgcn_perm(0x00000001u, 0x0000FF00u, w & 0x0C0C0C0Cu));
}

__device__ __forceinline__ v4i t2_unpack(uint32_t word) {
    const uint32_t hi = word >> 4;
    return v4i{t2_even(word), t2_odd(word), t2_even(hi), t2_odd(hi)};
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
    v4i v[2][4];
};
template <>
struct AFrag<kDenseT2> {
    v4i h[2];  // half h, word j: row block 2h + j/2, k-tile j % 2
};

// NB = 16-trial blocks per workgroup (trial tile = 16 NB).  MODE: what every
// run of the launch is -- kDenseAny: tested at run time; kDensePlain: pSA with
// one sub-step per step (no held inputs, windows or periods), so the epilogue
// carries no run-time mode tests; kDenseIdentity: that, and every p-bit has
// lambda = 1, delta = 0 and no timing gate, so the pre-activation is the one
// product I0 (float)L (exactly the general (I0 lambda)((float)L + delta) at
// those values) and no gate word is drawn.
enum : int { kDenseAny = 0, kDensePlain = 1, kDenseIdentity = 2 };
template <int NB, int ENC, int MODE>
__global__ __launch_bounds__(256, ENC == kDenseT2 ? 3 : 2) void dense_step_kernel(const DenseJob *__restrict__ jobs,
                                                         const int4 *__restrict__ work, int32_t t_off) {
    constexpr bool PLAIN = MODE != kDenseAny;
    constexpr int kTrials = 16 * NB;
    constexpr int kBVec = kTrials * (kKC / 16);        // 16-byte pieces of one spin chunk
    constexpr int kBPer = (kBVec + 255) / 256;  // 1 or 2
    __shared__ __align__(16) int8_t bt[2][kTrials * kLdsStride];
    const int4 w = work[blockIdx.x];  // (job, row group, trial tile, -); job < 0: empty slot
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
    auto fetch_b = [&](int kc) {
        breg0 = *as_global<v4i>(gcur + static_cast<size_t>(trial0 + (c0 >> 3)) * np + kc * kKC + (c0 & 7) * 16);
        if constexpr (kBPer == 2) {
            const int c = c0 + 256;
            breg1 = *as_global<v4i>(gcur + static_cast<size_t>(trial0 + (c >> 3)) * np + kc * kKC + (c & 7) * 16);
        }
    };
    auto store_b = [&](int buf) {
        *reinterpret_cast<v4i *>(&bt[buf][(c0 >> 3) * kLdsStride + (c0 & 7) * 16]) = breg0;
        if constexpr (kBPer == 2) {
            const int c = c0 + 256;
            *reinterpret_cast<v4i *>(&bt[buf][(c >> 3) * kLdsStride + (c & 7) * 16]) = breg1;
        }
    };
    auto fetch_a = [&](int kc, AFrag<ENC> &dst) {
        if constexpr (ENC == kDenseI8) {
            const gptr<int8_t> J = as_global<int8_t>(jb.J);
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const size_t row = static_cast<size_t>(arow0 + rb * 16 + lr);
                    dst.v[kt][rb] = *as_global<v4i>(J + row * np + kc * kKC + kt * 64 + kgrp);
                }
        } else {
            const gptr<v4i> J = as_global<v4i>(jb.J);
            const size_t tile = (static_cast<size_t>(arow0 / kWaveRows) * (np / kKC) + kc) * 2;
            dst.h[0] = J[tile * 64 + lane];
            dst.h[1] = J[(tile + 1) * 64 + lane];
        }
    };

    v4i acc[4][NB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = v4i{0, 0, 0, 0};

    auto compute = [&](int buf, const AFrag<ENC> &af) {
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            v4i b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                b[nb] = *reinterpret_cast<const v4i *>(&bt[buf][(nb * 16 + lr) * kLdsStride + kt * 64 + kgrp]);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                v4i a;
                if constexpr (ENC == kDenseI8)
                    a = af.v[kt][rb];
                else
                    a = t2_unpack(static_cast<uint32_t>(af.h[rb >> 1][(rb & 1) * 2 + kt]));
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[rb][nb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b[nb], acc[rb][nb], 0, 0, 0);
            }
        }
    };
    const int nkc = np / kKC;
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
    // nb.
    const float i0t = jb.i0[t];
    if constexpr (MODE == kDenseIdentity) {
        // one r block and four products per (row block, trial block) pair; the
        // pairs unrolled with constant accumulator indices, a scheduling
        // barrier between them keeping one pair's temporaries live at a time
        const int32_t scale = jb.scale;
        const uint32_t kpos = static_cast<uint32_t>(trial0 + lr);
#pragma unroll
        for (int e = 0; e < 4 * NB; ++e) {
            const int rb = e / NB, nb = e % NB;
            const int32_t i0 = wrow0 + rb * 16 + (lane >> 4) * 4;
            const uint32_t k = kpos + static_cast<uint32_t>(nb * 16);
            const bool valid = i0 < jb.n4 && static_cast<int32_t>(k) < jb.t4;
            const int4 hh = *reinterpret_cast<const int4 *>(jb.h + (valid ? i0 : 0));
            const Words4 r = philox4x32_10(tau, static_cast<uint32_t>(i0 >> 2), k, kTagR, jb.k0, jb.k1);
            const int32_t hv[4] = {hh.x, hh.y, hh.z, hh.w};
            const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
            uint32_t out = 0u;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int32_t L = hv[p] + scale * acc[rb][nb][p];
                const float x = i0t * static_cast<float>(L);
                out |= (pbit_up(x, rw[p]) ? 0x01u : 0xFFu) << (8 * p);
            }
            if (valid) *reinterpret_cast<uint32_t *>(nxt + static_cast<size_t>(k) * np + i0) = out;
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    // the other modes: the (row block, trial block) pairs run as a loop with a
    // uniform index, so the body -- Philox blocks and four activations -- is
    // emitted once per pass, keeping few registers live.
    const int32_t scale = jb.scale;
    const InputState st{jb.xs, jb.stall24, jb.ring, jb.alpha, jb.n4};
    auto update = [&](int e, const v4i a4) __attribute__((always_inline)) {
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
            old = *reinterpret_cast<const uint32_t *>(cur + static_cast<size_t>(k) * np + i0);
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
        uint32_t out = 0u;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int32_t L = hv[p] + scale * a4[p];
            const float x = PLAIN ? input_of<kAlgPsa>(av[p], dv[p], L, sv, i0 + p, static_cast<uint32_t>(k),
                                                      static_cast<uint32_t>(t), sw[p])
                                  : input_any(av[p], dv[p], L, sv, i0 + p, static_cast<uint32_t>(k),
                                      static_cast<uint32_t>(t), sw[p]);
            const bool up = pbit_up(x, rw[p]);
            const bool fire = period_mode ? period_fires(tau, tv[p])
                                          : (tv[p] >= kGateOne || fires(gw[p], tv[p]));
            const uint32_t ob = (old >> (8 * p)) & 0xFFu;
            out |= (fire ? (up ? 0x01u : 0xFFu) : ob) << (8 * p);
        }
        if (valid) *reinterpret_cast<uint32_t *>(nxt + static_cast<size_t>(k) * np + i0) = out;
    };
    // The accumulators move through a queue read only at its head (constant
    // register indices; a loop index into the array would force it into
    // scratch memory).  Two (row block, trial block) pairs per pass: their
    // Philox chains are independent, which doubles the instruction-level
    // parallelism.
    v4i q[4 * NB];
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

// [n][t4] (trials innermost) <-> [tp][np] (p-bits contiguous); padding
// p-bits and trials of the dense layout are +1.
__global__ void to_dense_kernel(int32_t n, int32_t t4, int32_t np, int32_t tp,
                                const int8_t *__restrict__ spins, int8_t *__restrict__ m) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(tp) * np) return;
    const int32_t k = static_cast<int32_t>(idx / np);
    const int32_t i = static_cast<int32_t>(idx % np);
    m[idx] = (i < n && k < t4) ? spins[static_cast<size_t>(i) * t4 + k] : int8_t(1);
}

__global__ void from_dense_kernel(int32_t n, int32_t t4, int32_t np, const int8_t *__restrict__ m,
                                  int8_t *__restrict__ spins) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * t4) return;
    const int32_t i = static_cast<int32_t>(idx / t4);
    const int32_t k = static_cast<int32_t>(idx % t4);
    spins[idx] = m[static_cast<size_t>(k) * np + i];
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
        const hipError_t e = enc == kDenseT2 ? launch_dense_mode<kDenseT2>(stream, jobs, work, nwork, nb, mode, s)
                                             : launch_dense_mode<kDenseI8>(stream, jobs, work, nwork, nb, mode, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_to_dense(hipStream_t stream, int32_t n, int32_t t4, int32_t np, int32_t tp,
                           const int8_t *spins, int8_t *m) {
    const int64_t items = static_cast<int64_t>(tp) * np;
    hipLaunchKernelGGL(to_dense_kernel, dim3(static_cast<unsigned>((items + 255) / 256)), dim3(256), 0,
                       stream, n, t4, np, tp, spins, m);
    return hipGetLastError();
}

hipError_t launch_from_dense(hipStream_t stream, int32_t n, int32_t t4, int32_t np,
                             const int8_t *m, int8_t *spins) {
    const int64_t items = static_cast<int64_t>(n) * t4;
    hipLaunchKernelGGL(from_dense_kernel, dim3(static_cast<unsigned>((items + 255) / 256)), dim3(256),
                       0, stream, n, t4, np, m, spins);
    return hipGetLastError();
}

}  // namespace psa
