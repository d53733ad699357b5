// device_math.hpp -- per-update arithmetic of the p-bit (gfx950 device code).
//
// Counter-based randomness, the uniform r of Eq. 1, the timing gate, and a
// single-precision tanh with a fixed operation order.  Every value here is
// evaluated with IEEE single-precision operations that round exactly once
// (explicit fmaf, correctly rounded division, no contraction), so that the
// result does not depend on how the compiler schedules it; the decision
// pbit_up takes hardware approximations only where they cannot change it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psa {

// Purposes of the random words; part of the Philox counter.
enum : uint32_t { kTagInit = 0, kTagR = 1, kTagGate = 2, kTagVar = 3, kTagStall = 4 };

constexpr uint32_t kGateOne = 1u << 24;

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by M0 = 0xD2511F53 and M1 = 0xCD9E8D57, with the key
// advanced by the Weyl increments W0 = 0x9E3779B9, W1 = 0xBB67AE85 between
// rounds.  Returns the four output words in (x, y, z, w).
struct Words4 {
    uint32_t x, y, z, w;
};

// State of one block between rounds: counter words and the round's key.
struct PhiloxState {
    uint32_t c0, c1, c2, c3, k0, k1;
};

// R more rounds of the block (a caller may split the ten rounds to place
// them between other work).
template <int R>
__device__ __forceinline__ void philox_rounds(PhiloxState &s) {
#pragma unroll
    for (int round = 0; round < R; ++round) {
        // one 32x32->64 multiply-add instruction per product on gfx950
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * s.c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * s.c2;
        // three-input XOR in one instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), s.c1, s.k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), s.c3, s.k1, 0x96);
        s.c1 = static_cast<uint32_t>(p1);
        s.c3 = static_cast<uint32_t>(p0);
        s.c0 = n0;
        s.c2 = n2;
        s.k0 += 0x9E3779B9u;
        s.k1 += 0xBB67AE85u;
    }
}

// The block's starting state; the key is uniform (one per run) and lives in
// scalar registers, kept opaque here so that its schedule is formed on the
// scalar unit at each use rather than hoisted out of the loops into spilled
// registers.
__device__ __forceinline__ PhiloxState philox_start(uint32_t c0, uint32_t c1, uint32_t c2,
                                                    uint32_t c3, uint32_t k0, uint32_t k1) {
    asm volatile("" : "+s"(k0), "+s"(k1));
    return PhiloxState{c0, c1, c2, c3, k0, k1};
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1,
                                                uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    PhiloxState s = philox_start(c0, c1, c2, c3, k0, k1);
    philox_rounds<10>(s);
    return Words4{s.c0, s.c1, s.c2, s.c3};
}

// The key schedule of one run (the key of each of the ten rounds), formed
// once by a kernel that draws many blocks under that key.
struct PhiloxKeys {
    uint32_t k0[10], k1[10];
};
__device__ __forceinline__ PhiloxKeys philox_keys(uint32_t k0, uint32_t k1) {
    PhiloxKeys K;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        K.k0[round] = k0;
        K.k1[round] = k1;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return K;
}
// The same ten rounds as philox4x32_10, each under its precomputed key.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                const PhiloxKeys &K) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, K.k0[round], 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, K.k1[round], 0x96);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
    }
    return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word_of(const Words4 &w, uint32_t k) {
    return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// Exchange a value with the neighbouring lane of the pair (lane ^ 1):
// DPP quad permutation [1, 0, 3, 2].  Both lanes of a pair must be active.
__device__ __forceinline__ uint32_t swap_pair(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0xB1, 0xF, 0xF, false));
}

// r in (-1, 1): the odd multiple of 2^-24 given by the top 25 bits of a word
// with the lowest forced to one, ((u >> 7) | 1) 2^-24 - 1 = (u >> 8) 2^-23 +
// 2^-24 - 1: the 24-bit integer converts exactly and the single fma rounds
// nothing (its result is representable).
__device__ __forceinline__ float r_of(uint32_t u) {
    return fmaf(static_cast<float>(u >> 8), 0x1p-23f, 0x1p-24f - 1.0f);
}

// Timing gate for a p-bit whose update probability is thr24 / 2^24 (< 1).
__device__ __forceinline__ bool fires(uint32_t u, uint32_t thr24) {
    return (u >> 8) < thr24;
}

// tanh(x) = sign(x) (1 - 2 / (e^{2|x|} + 1)); e^{2|x|} = 2^v, v = 2|x| log2 e,
// split v = n + f (n nearest integer, |f| <= 1/2); 2^f from the degree-7
// Taylor polynomial of e^{f ln 2} (coefficients (ln 2)^k / k!, rounded to
// float), Horner with fused multiply-add; |x| >= 9 gives exactly +-1.
__device__ __forceinline__ float tanh_f32(float x) {
    const float a = fminf(fabsf(x), 9.0f);
    const float v = a * 0x1.715476p+1f;
    const float nf = rintf(v);
    const float f = v - nf;
    float p = 0x1.ffcbfcp-17f;
    p = fmaf(p, f, 0x1.430912p-13f);
    p = fmaf(p, f, 0x1.5d87fep-10f);
    p = fmaf(p, f, 0x1.3b2ab6p-7f);
    p = fmaf(p, f, 0x1.c6b08ep-5f);
    p = fmaf(p, f, 0x1.ebfbe0p-3f);
    p = fmaf(p, f, 0x1.62e430p-1f);
    p = fmaf(p, f, 1.0f);
    const float e = ldexpf(p, static_cast<int>(nf));
    float y = 1.0f - 2.0f / (e + 1.0f);
    y = (a >= 9.0f) ? 1.0f : y;
    return copysignf(y, x);
}

// Eq. 1 decision: +1 iff tanh_f32(x) > r.  A cheap estimate of tanh (the
// hardware 2^v and reciprocal, each within about one ulp, in place of the
// polynomial and the correctly rounded division) decides whenever it lies
// more than 2^-16 from r.  The estimate is within 2^-20 of tanh_f32(x): a
// relative error of about 2^-21 in 2^v moves 1 - 2/(e+1) by at most half
// that, the reciprocal adds 2^-23 and the roundings a few 2^-24; so every
// such decision is the one tanh_f32 gives.  The rest (about 2^-16 of the
// updates) evaluate tanh_f32 itself.
__device__ __forceinline__ float tanh_estimate_minus(float x, float r) {
    const float a = fminf(fabsf(x), 9.0f);
    const float e = __builtin_amdgcn_exp2f(a * 0x1.715476p+1f);
    const float y = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
    return copysignf(y, x) - r;
}

// True when the estimate's distance to r decides (else tanh_f32 is evaluated).
__device__ __forceinline__ bool estimate_decides(float diff) { return fabsf(diff) > 0x1p-16f; }

__device__ __forceinline__ bool pbit_up(float x, uint32_t rword) {
    const float r = r_of(rword);
    const float diff = tanh_estimate_minus(x, r);
    if (estimate_decides(diff)) return diff > 0.0f;
    return tanh_f32(x) > r;
}

// 16-byte load from device-global memory through an address-space cast, so
// that it is issued as a global (not flat) load and does not wait on LDS
// traffic.  p must be 16-byte aligned.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 load_global_x4(const void *p) {
    return *(const u32x4 __attribute__((address_space(1))) *)(p);
}

// Input-stage state of one run (Eq. 4 / Eq. 5 variants), both laid out as
// [t4/4][n4] x (trial in group innermost):
//   xs    SpSA held pre-activations, [t4/4][n4][4] floats (else nullptr);
//   ring  TApSA field windows, [t4/4][n4][alpha][4] int32 (else nullptr).
struct InputState {
    float *xs;
    uint32_t s24;
    int32_t *ring;
    int32_t alpha;
    int32_t n4;
};

// Input / timing variants of the sweep: plain pSA, SpSA, TApSA, and plain pSA
// with period-mode timing.
enum : int { kAlgPsa = 0, kAlgSpsa = 1, kAlgTapsa = 2, kAlgPeriod = 3 };

// Period mode: does a p-bit of period P (0 = never) fire at sub-step tau?
// tau < 2^22, so the quotient from a float reciprocal is within one of
// tau / P and one correction each way gives the exact remainder.
__device__ __forceinline__ bool period_fires(uint32_t tau, uint32_t P) {
    if (P == 0u) return false;
    const float fq = static_cast<float>(tau) * __builtin_amdgcn_rcpf(static_cast<float>(P));
    int32_t r = static_cast<int32_t>(tau) - static_cast<int32_t>(fq) * static_cast<int32_t>(P);
    if (r < 0) r += static_cast<int32_t>(P);
    if (r >= static_cast<int32_t>(P)) r -= static_cast<int32_t>(P);
    return r == 0;
}

// Input stage of p-bit i, trial k at step t, on the field L of step t; a =
// I0 lambda_i, d = delta_i.
//   pSA   (Eq. 3): x = a (L + d).
//   SpSA  (Eq. 5): the input is held from the last refresh iff t > 0 and
//         (stall word >> 8) < stall24, else formed anew as above and stored.
//   TApSA (Eq. 4): L enters the window slot t mod alpha; x = a (mean + d),
//         mean = (float)sum / (float)count over the last min(t+1, alpha)
//         fields.
template <int ALG>
__device__ __forceinline__ float input_of(float a, float d, int32_t L, const InputState &st,
                                          int32_t i, uint32_t k, uint32_t t, uint32_t sword) {
    if constexpr (ALG == kAlgSpsa) {
        const float x = a * (static_cast<float>(L) + d);
        float *slot = st.xs + ((static_cast<size_t>(k >> 2) * st.n4 + i) * 4 + (k & 3u));
        if (t > 0 && (sword >> 8) < st.s24) return *slot;
        *slot = x;
        return x;
    } else if constexpr (ALG == kAlgTapsa) {
        const uint32_t al = static_cast<uint32_t>(st.alpha);
        int32_t *w = st.ring + (static_cast<size_t>(k >> 2) * st.n4 + i) * al * 4 + (k & 3u);
        w[(t % al) * 4] = L;
        const uint32_t count = t + 1 < al ? t + 1 : al;
        int32_t sum = L;
        for (uint32_t q = 1; q < count; ++q) sum += w[((t - q) % al) * 4];
        const float mean = static_cast<float>(sum) / static_cast<float>(count);
        return a * (mean + d);
    } else {
        (void)st, (void)i, (void)k, (void)t, (void)sword;
        return a * (static_cast<float>(L) + d);
    }
}

// The same with the variant chosen at run time from the state pointers.
__device__ __forceinline__ float input_any(float a, float d, int32_t L, const InputState &st,
                                           int32_t i, uint32_t k, uint32_t t, uint32_t sword) {
    if (st.ring != nullptr) return input_of<kAlgTapsa>(a, d, L, st, i, k, t, sword);
    if (st.xs != nullptr) return input_of<kAlgSpsa>(a, d, L, st, i, k, t, sword);
    return input_of<kAlgPsa>(a, d, L, st, i, k, t, sword);
}

// Sign-extend byte k of a packed word of four int8 spins.
__device__ __forceinline__ int32_t spin_of(uint32_t word, int k) {
    return static_cast<int32_t>(word << (24 - 8 * k)) >> 24;
}

}  // namespace psa
