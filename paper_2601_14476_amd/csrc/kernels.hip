// kernels.hip -- gfx950 kernels of the pSA hot path.
//
//   init_spins_kernel   initial state: m = +1 iff bit 31 of the INIT word
//   local_field_kernel  L = h + J m (Eq. 3 without I0), for tests
//   energy_partial_kernel, energy_finish_kernel   Eq. 2 energy and MAX-CUT value per trial
//   spins_{to,from}_tn  layout conversion [n][t4] <-> [trials][n]
//
// (The persistent sweep kernel is in anneal.hip.)  Random words: Philox4x32-10
// block of counter (t, i/4, k, purpose) serves the four p-bits 4m..4m+3
// (m = i/4) of trial k; word i mod 4.
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

// Pass 1: workgroup (row block, trial group q) sums, over its 256 rows, the
// row terms m_i sum_j J_ij m_j and h_i m_i of the four trials of q; thread
// per row.  part[(block * groups + q) * 8 + c]: c < 4 the S terms of trial
// 4q + c, c >= 4 the h terms.
__device__ __forceinline__ void energy_partial(int32_t n, int32_t t4, const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col, const int32_t *__restrict__ val,
                                               const int32_t *__restrict__ h, const int8_t *__restrict__ spins,
                                               int64_t *__restrict__ part, int32_t blk, int32_t q) {
    const int32_t groups = t4 / 4;
    const int32_t i = blk * kEnergyBlock + threadIdx.x;
    int64_t s[4] = {0, 0, 0, 0};
    int64_t hm[4] = {0, 0, 0, 0};
    if (i < n) {
        const uint32_t wi = load_word(spins, t4, i, q);
        int32_t L[4] = {0, 0, 0, 0};
        const int32_t e1 = row_ptr[i + 1];
#pragma unroll 4
        for (int32_t e = row_ptr[i]; e < e1; ++e) {
            const uint32_t wj = load_word(spins, t4, col[e], q);
            const int32_t J = val[e];
#pragma unroll
            for (int k = 0; k < 4; ++k) L[k] += J * spin_of(wj, k);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t mi = spin_of(wi, k);
            s[k] = static_cast<int64_t>(mi * L[k]);
            hm[k] = static_cast<int64_t>(mi * h[i]);
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
    if (threadIdx.x < 8) {
        int64_t v = 0;
        for (int w = 0; w < kEnergyBlock / 64; ++w) v += red[w][threadIdx.x];
        part[(static_cast<size_t>(blk) * groups + q) * 8 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(kEnergyBlock) void energy_partial_kernel(
    int32_t n, int32_t t4, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ val, const int32_t *__restrict__ h,
    const int8_t *__restrict__ spins, int64_t *__restrict__ part) {
    energy_partial(n, t4, row_ptr, col, val, h, spins, part, blockIdx.x, blockIdx.y);
}

// Pass 2: thread per trial k sums the row blocks' terms:
//   E_k   = -sum_i h_i m_i - S_k / 2
//   cut_k = sum_{i<j} w_ij [m_i != m_j] = (S_k - W2) / 4     (w = -J)
__device__ __forceinline__ void energy_finish(int32_t blocks, int32_t groups, int32_t k, int64_t w2,
                                              const int64_t *__restrict__ part, int64_t *__restrict__ energy,
                                              int64_t *__restrict__ cut) {
    const int32_t q = k >> 2, c = k & 3;
    int64_t S = 0, H = 0;
    for (int32_t b = 0; b < blocks; ++b) {
        S += part[(static_cast<size_t>(b) * groups + q) * 8 + c];
        H += part[(static_cast<size_t>(b) * groups + q) * 8 + 4 + c];
    }
    energy[k] = -H - S / 2;
    cut[k] = (S - w2) / 4;
}

__global__ void energy_finish_kernel(int32_t blocks, int32_t groups, int32_t trials, int64_t w2,
                                     const int64_t *__restrict__ part, int64_t *__restrict__ energy,
                                     int64_t *__restrict__ cut) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= trials) return;
    energy_finish(blocks, groups, k, w2, part, energy, cut);
}

// The run of a batched read-out that index x (a workgroup of the partial
// pass, or a trial of the final pass) belongs to: the last run whose first
// index is at most x (first indices ascending, the first one 0).
template <bool WG>
__device__ __forceinline__ int32_t energy_run_of(const EnergyJob *__restrict__ jobs, int32_t count, int32_t x) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((WG ? jobs[mid].wg0 : jobs[mid].k0) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Batched partial pass, sixteen trials per lane: workgroup (row block, chunk
// y of four trial groups) sums the terms of groups 4y..4y+3 (those below
// t4 / 4) into the same part entries as energy_partial.  LPR lanes share a
// row: lane `sub` of a group takes the row's edges sub, sub + LPR, ... (so
// the group's column and coupling reads are contiguous), reading each edge's
// column and coupling once per 16 trials and, when t4 is a multiple of 16,
// the neighbour's 16 spins in one load.  Because S = sum_i m_i sum_j J_ij m_j
// is linear in each row's inner sum, every lane multiplies its share of the
// inner sum by m_i and keeps the products; the h terms are taken by lane 0 of
// the group.  A group's rows are g, g + 256 / LPR, ... of the block.  A row's
// terms are below 2^24 in magnitude (the field bound), so a lane's sum over
// its LPR <= 16 rows fits int32; sums across lanes are taken in int64.
constexpr int kEnergyQuads = 4;

template <int LPR>
__device__ __forceinline__ void energy_partial16(const EnergyJob &e, int32_t blk, int32_t y) {
    constexpr int Q = kEnergyQuads;
    constexpr int kGroups = kEnergyBlock / LPR;
    const int32_t t4 = e.t4;
    const int32_t groups = t4 / 4;
    const int32_t q0 = y * Q;
    const int32_t nq = groups - q0 < Q ? groups - q0 : Q;  // workgroup-uniform
    const bool vec = (t4 & 15) == 0 && (reinterpret_cast<uintptr_t>(e.spins) & 15) == 0;
    const int32_t sub = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    int32_t s32[Q][4] = {}, hm32[Q][4] = {};
    for (int32_t r = 0; r < LPR; ++r) {
        const int32_t i = blk * kEnergyBlock + grp + kGroups * r;
        if (i >= e.n) break;
        int32_t L[Q][4] = {};
        const int32_t e1 = e.row_ptr[i + 1];
#pragma unroll 2
        for (int32_t x = e.row_ptr[i] + sub; x < e1; x += LPR) {
            const int32_t j = e.col[x];
            const int32_t J = e.val[x];
            uint32_t w[Q] = {0u, 0u, 0u, 0u};
            if (vec) {
                const uint4 v4 = *reinterpret_cast<const uint4 *>(e.spins + static_cast<size_t>(j) * t4 + 4 * q0);
                w[0] = v4.x;
                w[1] = v4.y;
                w[2] = v4.z;
                w[3] = v4.w;
            } else {
#pragma unroll
                for (int qq = 0; qq < Q; ++qq)
                    if (qq < nq) w[qq] = load_word(e.spins, t4, j, q0 + qq);
            }
#pragma unroll
            for (int qq = 0; qq < Q; ++qq)
#pragma unroll
                for (int k = 0; k < 4; ++k) L[qq][k] += J * spin_of(w[qq], k);
        }
        const int32_t hi = sub == 0 ? e.h[i] : 0;
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) {
            if (qq < nq) {
                const uint32_t wi = load_word(e.spins, t4, i, q0 + qq);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t mi = spin_of(wi, k);
                    s32[qq][k] += mi * L[qq][k];
                    hm32[qq][k] += mi * hi;
                }
            }
        }
    }
    int64_t s[Q][4], hm[Q][4];
#pragma unroll
    for (int qq = 0; qq < Q; ++qq)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[qq][k] = s32[qq][k];
            hm[qq][k] = hm32[qq][k];
        }
    __shared__ int64_t red[kEnergyBlock / 64][Q][8];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int qq = 0; qq < Q; ++qq)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            for (int off = 32; off > 0; off >>= 1) {
                s[qq][k] += __shfl_down(s[qq][k], off, 64);
                hm[qq][k] += __shfl_down(hm[qq][k], off, 64);
            }
    if (lane == 0) {
#pragma unroll
        for (int qq = 0; qq < Q; ++qq)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                red[wave][qq][k] = s[qq][k];
                red[wave][qq][4 + k] = hm[qq][k];
            }
    }
    __syncthreads();
    if (threadIdx.x < 8 * Q) {
        const int qq = threadIdx.x >> 3, c = threadIdx.x & 7;
        if (qq < nq) {
            int64_t v = 0;
            for (int wv = 0; wv < kEnergyBlock / 64; ++wv) v += red[wv][qq][c];
            e.part[(static_cast<size_t>(blk) * groups + q0 + qq) * 8 + c] = v;
        }
    }
}

// Batched partial pass: workgroup b is (row block, chunk of four trial
// groups) b - wg0 of its run, row block major; the run's lanes per row
// (1, 4 or 16) pick the variant, uniform over the workgroup.
__global__ __launch_bounds__(kEnergyBlock) void energy_partial_batch_kernel(const EnergyJob *__restrict__ jobs,
                                                                            int32_t count) {
    const int32_t b = blockIdx.x;
    const EnergyJob &e = jobs[energy_run_of<true>(jobs, count, b)];
    const int32_t chunks = (e.t4 / 4 + kEnergyQuads - 1) / kEnergyQuads;
    const int32_t local = b - e.wg0;
    if (e.lpr >= 16)
        energy_partial16<16>(e, local / chunks, local % chunks);
    else if (e.lpr >= 4)
        energy_partial16<4>(e, local / chunks, local % chunks);
    else
        energy_partial16<1>(e, local / chunks, local % chunks);
}

// Batched final pass: thread x is trial x - k0 of its run.
__global__ void energy_finish_batch_kernel(const EnergyJob *__restrict__ jobs, int32_t count, int32_t trials) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= trials) return;
    const EnergyJob &e = jobs[energy_run_of<false>(jobs, count, x)];
    energy_finish(e.blocks, e.t4 / 4, x - e.k0, e.w2, e.part, e.energy, e.cut);
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

// ---------------------------------------------------------------------------
// Value-level checks of the per-update arithmetic (test entry points): the
// device tanh_f32 of every x, and the decision pbit_up of every (x, word)
// with the branch it took (bit 0: +1, bit 1: the estimate was within 2^-16
// of r, so tanh_f32 decided).  Grid-stride over count elements.
// ---------------------------------------------------------------------------
__global__ void debug_tanh_kernel(int64_t count, const float *__restrict__ x,
                                  float *__restrict__ y) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += stride)
        y[i] = tanh_f32(x[i]);
}

__global__ void debug_decide_kernel(int64_t count, const float *__restrict__ x,
                                    const uint32_t *__restrict__ word, uint8_t *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += stride) {
        const float diff = tanh_estimate_minus(x[i], r_of(word[i]));
        out[i] = static_cast<uint8_t>((pbit_up(x[i], word[i]) ? 1u : 0u) |
                                      (estimate_decides(diff) ? 0u : 2u));
    }
}

}  // namespace

hipError_t launch_init_spins(hipStream_t stream, int32_t n, const DevRun &run) {
    const int32_t tasks = (n + 3) / 4;
    const int block = 256;
    hipLaunchKernelGGL(init_spins_kernel, dim3(grid_for(static_cast<int64_t>(tasks) * run.t4, block)),
                       dim3(block), 0, stream, n, tasks, run.t4, run.key0, run.key1, run.spins);
    return hipGetLastError();
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

size_t energy_partial_bytes(int32_t n, int32_t t4) {
    return static_cast<size_t>((n + kEnergyBlock - 1) / kEnergyBlock) * (t4 / 4) * 8 * sizeof(int64_t);
}

hipError_t launch_energy_cut(hipStream_t stream, const DevGraph &g, const DevRun &run,
                             int64_t *part, int64_t *energy, int64_t *cut) {
    const int32_t blocks = (g.n + kEnergyBlock - 1) / kEnergyBlock;
    const int32_t groups = run.t4 / 4;
    hipLaunchKernelGGL(energy_partial_kernel, dim3(blocks, groups), dim3(kEnergyBlock), 0, stream,
                       g.n, run.t4, g.row_ptr, g.col, g.val, g.h, run.spins, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_finish_kernel, dim3(grid_for(run.trials, 256)), dim3(256), 0, stream,
                       blocks, groups, run.trials, g.w2, part, energy, cut);
    return hipGetLastError();
}

hipError_t launch_energy_cut_batch(hipStream_t stream, const EnergyJob *jobs, int32_t count, int32_t wgs,
                                   int32_t trials) {
    if (count <= 0 || wgs <= 0 || trials <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_partial_batch_kernel, dim3(wgs), dim3(kEnergyBlock), 0, stream, jobs, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_finish_batch_kernel, dim3(grid_for(trials, 256)), dim3(256), 0, stream, jobs, count,
                       trials);
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

hipError_t launch_debug_tanh(hipStream_t stream, int64_t count, const float *x, float *y) {
    const int block = 256;
    const int64_t grid = std::min<int64_t>((count + block - 1) / block, 8192);
    hipLaunchKernelGGL(debug_tanh_kernel, dim3(static_cast<uint32_t>(grid)), dim3(block), 0, stream,
                       count, x, y);
    return hipGetLastError();
}

hipError_t launch_debug_decide(hipStream_t stream, int64_t count, const float *x,
                               const uint32_t *word, uint8_t *out) {
    const int block = 256;
    const int64_t grid = std::min<int64_t>((count + block - 1) / block, 8192);
    hipLaunchKernelGGL(debug_decide_kernel, dim3(static_cast<uint32_t>(grid)), dim3(block), 0,
                       stream, count, x, word, out);
    return hipGetLastError();
}

}  // namespace psa
