// densify.hip -- the densification step around the renderer (Sec. 3.2,
// "Densification"): Bernoulli sampling of triangles with probabilities from
// their opacity or inverse sigma, and midpoint subdivision of the selected
// ones in place.  Per-triangle streaming kernels, bound by HBM.
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kDensBlock = 256;
constexpr int kSumChunk = 4096;   // weights per workgroup of the partial sums

__device__ __forceinline__ double dens_weight(const float* __restrict__ o,
                                              const float* __restrict__ sigma, int mode, int64_t i)
{
    return mode == TS_DENSIFY_OPACITY ? (double)o[i] : 1.0 / (double)sigma[i];
}

// Sum of 256 doubles in LDS by a fixed tree: the result does not depend on
// timing, so the sum (and every decision taken from it) is reproducible.
__device__ __forceinline__ double block_sum(double x, double* s)
{
    const int t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (int h = kDensBlock / 2; h > 0; h >>= 1) {
        if (t < h) s[t] += s[t + h];
        __syncthreads();
    }
    return s[0];
}

__global__ __launch_bounds__(kDensBlock) void k_weight_partial(
    const float* __restrict__ o, const float* __restrict__ sigma, int64_t N, int mode,
    double* __restrict__ partial)
{
    __shared__ double s[kDensBlock];
    const int64_t base = (int64_t)blockIdx.x * kSumChunk;
    double acc = 0.0;
    for (int j = threadIdx.x; j < kSumChunk; j += kDensBlock) {
        const int64_t i = base + j;
        if (i < N) acc += dens_weight(o, sigma, mode, i);
    }
    const double tot = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kDensBlock) void k_weight_total(const double* __restrict__ partial,
                                                             int64_t nb, double* __restrict__ total)
{
    __shared__ double s[kDensBlock];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < nb; j += kDensBlock) acc += partial[j];
    const double tot = block_sum(acc, s);
    if (threadIdx.x == 0) total[0] = tot;
}

// p_i = min(1, k w_i / sum w); selected iff u_i < p_i (all in FP64).
__global__ __launch_bounds__(kDensBlock) void k_select(
    const float* __restrict__ o, const float* __restrict__ sigma, int64_t N, int mode, double k,
    const double* __restrict__ total, const float* __restrict__ u, uint8_t* __restrict__ sel)
{
    const int64_t i = (int64_t)blockIdx.x * kDensBlock + threadIdx.x;
    if (i >= N) return;
    const double tot = total[0];
    const double p = tot > 0.0 ? fmin(1.0, k * dens_weight(o, sigma, mode, i) / tot) : 0.0;
    sel[i] = (double)u[i] < p ? 1 : 0;
}

// Per-workgroup count of selected triangles.
__global__ __launch_bounds__(kDensBlock) void k_count_sel(const uint8_t* __restrict__ sel,
                                                          int64_t N, uint32_t* __restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * kDensBlock + threadIdx.x;
    const int c = __syncthreads_count(i < N && sel[i] != 0);
    if (threadIdx.x == 0) cnt[blockIdx.x] = (uint32_t)c;
}

// Exclusive scan of the per-workgroup counts by one workgroup of 1024
// threads, 1024 counts per round (coalesced loads, wave scans by shuffles,
// one LDS exchange of the 16 wave sums); out[0] = N + 3 n (the new count),
// out[1] = 1 when that exceeds the capacity (then nothing is written).
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan_sel(uint32_t* __restrict__ cnt,
                                                           int64_t nb, int64_t N,
                                                           int64_t capacity,
                                                           uint32_t* __restrict__ out)
{
    __shared__ uint32_t ws[kScanThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    uint64_t run = 0;   // the same in every thread
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t j = base + t;
        const uint32_t x = j < nb ? cnt[j] : 0u;
        uint32_t v = x;   // inclusive scan over the wave
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(v, o);
            v += lane >= o ? y : 0u;
        }
        if (lane == kWave - 1) ws[w] = v;
        __syncthreads();
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < kScanThreads / kWave; ++k) {
            const uint32_t sk = ws[k];
            before += k < w ? sk : 0u;
            tot += sk;
        }
        if (j < nb) cnt[j] = (uint32_t)(run + before + v - x);
        run += tot;
        __syncthreads();   // the wave sums are rewritten next round
    }
    if (t == 0) {
        const uint64_t total = (uint64_t)N + 3 * run;
        out[0] = (uint32_t)min(total, (uint64_t)0xffffffffu);
        out[1] = total > (uint64_t)capacity ? 1u : 0u;
    }
}

// Midpoint subdivision in place: the centre child replaces the parent, the
// three corner children go to N + 3 r + {0, 1, 2}, r the rank of the
// parent among the selected triangles; they copy its opacity, sigma and SH
// row.  Midpoints are (a + b) * 0.5 in FP32: one rounding.
__global__ __launch_bounds__(kDensBlock) void k_subdivide(
    float* __restrict__ v, float* __restrict__ o, float* __restrict__ sigma, float* __restrict__ sh,
    int nsh, int64_t N, const uint8_t* __restrict__ sel, const uint32_t* __restrict__ off,
    const uint32_t* __restrict__ out)
{
    __shared__ uint32_t s_w[kDensBlock / kWave];
    if (out[1] != 0u) return;   // does not fit: leave the soup unchanged
    const int64_t i = (int64_t)blockIdx.x * kDensBlock + threadIdx.x;
    const bool vec = (nsh & 3) == 0 && (reinterpret_cast<uintptr_t>(sh) & 15u) == 0;
    const bool me = i < N && sel[i] != 0;
    const uint64_t m = __ballot(me);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (lane == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0;
    for (int j = 0; j < w; ++j) before += s_w[j];
    const int64_t r = (int64_t)off[blockIdx.x] + before + below;
    if (vec) {
        // SH rows of whole 16-byte vectors (degrees 1 and 3): the wave copies
        // each selected lane's row to its three corner children together --
        // they are consecutive, so one wave store covers 3 rows contiguously
        const int n4 = nsh / 4;
        uint64_t todo = m;
        while (todo) {
            const int L = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t src_i = __shfl(i, L), dst_r = __shfl(r, L);
            const float4* s4 = reinterpret_cast<const float4*>(sh + (int64_t)nsh * src_i);
            float4* d4 = reinterpret_cast<float4*>(sh + (int64_t)nsh * (N + 3 * dst_r));
            for (int q = lane; q < 3 * n4; q += kWave) d4[q] = s4[q % n4];
        }
    }
    if (!me) return;

    float p[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) p[a] = v[9 * i + a];
    float m01[3], m12[3], m20[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m01[a] = (p[a] + p[3 + a]) * 0.5f;
        m12[a] = (p[3 + a] + p[6 + a]) * 0.5f;
        m20[a] = (p[6 + a] + p[a]) * 0.5f;
    }
    auto put = [&](int64_t j, const float* a0, const float* a1, const float* a2) {
        float* d = v + 9 * j;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d[a] = a0[a];
            d[3 + a] = a1[a];
            d[6 + a] = a2[a];
        }
    };
    put(i, m01, m12, m20);
    const int64_t j0 = N + 3 * r;
    put(j0, p, m01, m20);
    put(j0 + 1, m01, p + 3, m12);
    put(j0 + 2, m20, m12, p + 6);
    const float oi = o[i], si = sigma[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o[j0 + c] = oi;
        sigma[j0 + c] = si;
    }
    if (vec) return;   // copied by the wave above
    const float* src = sh + (int64_t)nsh * i;
    for (int q = 0; q < nsh; ++q) {
        const float x = src[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) sh[(int64_t)nsh * (j0 + c) + q] = x;
    }
}

size_t densify_workspace_bytes(int64_t N)
{
    const int64_t nw = (N + kSumChunk - 1) / kSumChunk, nb = (N + kDensBlock - 1) / kDensBlock;
    return (size_t)(8 * (nw + 1) + 4 * (nb + 2) + 256);
}

void launch_densify_select(const float* o, const float* sigma, int64_t N, int mode, double k,
                           const float* u, uint8_t* sel, void* ws, hipStream_t stream)
{
    const int64_t nw = (N + kSumChunk - 1) / kSumChunk, nb = (N + kDensBlock - 1) / kDensBlock;
    double* partial = reinterpret_cast<double*>(ws);
    double* total = partial + nw;
    hipLaunchKernelGGL(k_weight_partial, dim3((unsigned)nw), dim3(kDensBlock), 0, stream, o, sigma,
                       N, mode, partial);
    hipLaunchKernelGGL(k_weight_total, dim3(1), dim3(kDensBlock), 0, stream, partial, nw, total);
    hipLaunchKernelGGL(k_select, dim3((unsigned)nb), dim3(kDensBlock), 0, stream, o, sigma, N,
                       mode, k, total, u, sel);
}

void launch_densify_subdivide(float* v, float* o, float* sigma, float* sh, int nsh, int64_t N,
                              int64_t capacity, const uint8_t* sel, void* ws, uint32_t* d_out,
                              hipStream_t stream)
{
    const int64_t nb = (N + kDensBlock - 1) / kDensBlock;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(k_count_sel, dim3((unsigned)nb), dim3(kDensBlock), 0, stream, sel, N, cnt);
    hipLaunchKernelGGL(k_scan_sel, dim3(1), dim3(kScanThreads), 0, stream, cnt, nb, N, capacity,
                       d_out);
    hipLaunchKernelGGL(k_subdivide, dim3((unsigned)nb), dim3(kDensBlock), 0, stream, v, o, sigma,
                       sh, nsh, N, sel, cnt, d_out);
}

}  // namespace ts
