// dense.hip -- dense int8 matrix-core path of the local field (gfx950).
//
// For graphs whose rows are long, one synchronous step is a product of the
// dense coupling matrix with the spins of all trials,
//     L[i][k] = h_i + sum_j J_ij m_j,k      (int8 x int8 -> int32, exact),
// computed with v_mfma_i32_16x16x64_i8, followed by the p-bit update of
// Eq. 6 in the same kernel.  One launch advances one step of every dense run
// in a work list (run, 64-row tile, trial tile); the step loop is on the
// host (or in a captured graph of launches), because a step needs the whole
// previous state of its run.
//
// Layouts (per run):
//   J    int8 [np][np], np = n rounded up to 64, zero padding;
//   M    int8 [tp][np] per buffer (trial-major, p-bit index contiguous),
//        tp = trials rounded up to the trial tile; two buffers by step parity.
// MFMA operand layout (16x16x64, int8): lane l supplies A[row l%16][k (l/16)*16
// .. +15] and B[k (l/16)*16 .. +15][col l%16] as 16 bytes each, and receives
// D[row (l/16)*4 + r][col l%16] in its four accumulators r = 0..3.  The four
// rows of a lane are four consecutive p-bits 4m..4m+3 of one trial: exactly
// the p-bits one Philox block serves, so the epilogue draws one r block (and
// one gate block) per lane and trial column.
#include <hip/hip_runtime.h>

#include "device_math.hpp"
#include "engine.hpp"

namespace psa {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;            // rows per workgroup (4 waves x 16)
constexpr int kK = 64;               // K per MFMA
constexpr int kLdsStride = kK + 16;  // padded LDS row of the B tile (bytes)

__device__ __forceinline__ Words4 block_of(uint32_t t, uint32_t m, uint32_t k, uint32_t tag,
                                           uint32_t k0, uint32_t k1) {
    return philox4x32_10(t, m, k, tag, k0, k1);
}

// NB = 16-trial blocks per workgroup (trial tile = 16 NB).
template <int NB>
__global__ __launch_bounds__(256) void dense_step_kernel(const DenseJob *__restrict__ jobs,
                                                         const int4 *__restrict__ work, int32_t t_off) {
    __shared__ __align__(16) int8_t bt[2][16 * NB * kLdsStride];
    const int4 w = work[blockIdx.x];  // (job, row tile, trial tile, -)
    const DenseJob &jb = jobs[w.x];
    const int32_t t = jb.t + t_off;
    if (t >= jb.t_end) return;
    const int32_t np = jb.np;
    const int32_t row0 = w.y * kRows;
    const int32_t trial0 = w.z * (16 * NB);
    const int8_t *__restrict__ J = jb.J;
    const int8_t *__restrict__ cur = ((t - jb.t) & 1) ? jb.m1 : jb.m0;
    int8_t *__restrict__ nxt = ((t - jb.t) & 1) ? jb.m0 : jb.m1;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int arow = row0 + wave * 16 + (lane & 15);
    const int kgrp = (lane >> 4) * 16;

    v4i acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = v4i{0, 0, 0, 0};

    // cooperative B-tile load: 16*NB trial rows x 64 bytes, 16 bytes a thread
    auto load_b = [&](int buf, int k0) {
        for (int c = threadIdx.x; c < 16 * NB * 4; c += 256) {
            const int tr = c >> 2, part = (c & 3) * 16;
            const int4 v = *reinterpret_cast<const int4 *>(cur + static_cast<size_t>(trial0 + tr) * np + k0 + part);
            *reinterpret_cast<int4 *>(&bt[buf][tr * kLdsStride + part]) = v;
        }
    };
    load_b(0, 0);
    __syncthreads();
    const int nk = np / kK;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_b(buf ^ 1, (kt + 1) * kK);
        const v4i a = *reinterpret_cast<const v4i *>(J + static_cast<size_t>(arow) * np + kt * kK + kgrp);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const v4i b = *reinterpret_cast<const v4i *>(&bt[buf][(nb * 16 + (lane & 15)) * kLdsStride + kgrp]);
            acc[nb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[nb], 0, 0, 0);
        }
        __syncthreads();
    }

    // epilogue: lane owns p-bits 4m..4m+3 (m = task) for trial columns nb
    const int32_t i0 = row0 + wave * 16 + (lane >> 4) * 4;
    const int32_t m = i0 >> 2;
    if (i0 >= jb.n4) return;
    const float i0t = jb.i0[t];
    const int4 hh = *reinterpret_cast<const int4 *>(jb.h + i0);
    const uint4 th = *reinterpret_cast<const uint4 *>(jb.thr + i0);
    const float4 lm = *reinterpret_cast<const float4 *>(jb.lam + i0);
    const float4 dl = *reinterpret_cast<const float4 *>(jb.dlt + i0);
    const int32_t hv[4] = {hh.x, hh.y, hh.z, hh.w};
    const uint32_t tv[4] = {th.x, th.y, th.z, th.w};
    const float av[4] = {i0t * lm.x, i0t * lm.y, i0t * lm.z, i0t * lm.w};
    const float dv[4] = {dl.x, dl.y, dl.z, dl.w};
    const bool need_gate = (tv[0] < kGateOne) | (tv[1] < kGateOne) | (tv[2] < kGateOne) |
                           (tv[3] < kGateOne);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int32_t k = trial0 + nb * 16 + (lane & 15);
        if (k >= jb.t4) continue;
        const uint32_t old = *reinterpret_cast<const uint32_t *>(cur + static_cast<size_t>(k) * np + i0);
        uint32_t gw[4] = {0u, 0u, 0u, 0u};
        if (need_gate) {
            const Words4 g = block_of(static_cast<uint32_t>(t), static_cast<uint32_t>(m),
                                      static_cast<uint32_t>(k), kTagGate, jb.k0, jb.k1);
            gw[0] = g.x;
            gw[1] = g.y;
            gw[2] = g.z;
            gw[3] = g.w;
        }
        const Words4 r = block_of(static_cast<uint32_t>(t), static_cast<uint32_t>(m),
                                  static_cast<uint32_t>(k), kTagR, jb.k0, jb.k1);
        const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
        uint32_t out = 0u;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int32_t L = hv[p] + acc[nb][p];
            const float b = static_cast<float>(L) + dv[p];
            const float x = av[p] * b;
            const bool up = tanh_f32(x) > r_of(rw[p]);
            const bool fire = tv[p] >= kGateOne || fires(gw[p], tv[p]);
            const uint32_t ob = (old >> (8 * p)) & 0xFFu;
            out |= (fire ? (up ? 0x01u : 0xFFu) : ob) << (8 * p);
        }
        *reinterpret_cast<uint32_t *>(nxt + static_cast<size_t>(k) * np + i0) = out;
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

}  // namespace

hipError_t launch_dense_steps(hipStream_t stream, const DenseJob *jobs, const int4 *work,
                              int32_t nwork, int32_t nb, int32_t steps) {
    for (int32_t s = 0; s < steps; ++s) {
        switch (nb) {
            case 1: hipLaunchKernelGGL(dense_step_kernel<1>, dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
            case 2: hipLaunchKernelGGL(dense_step_kernel<2>, dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
            case 4: hipLaunchKernelGGL(dense_step_kernel<4>, dim3(nwork), dim3(256), 0, stream, jobs, work, s); break;
            default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
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
