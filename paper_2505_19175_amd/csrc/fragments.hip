// fragments.hip -- exclusive scan of the per-pixel fragment counts of the
// stored-fragment variant (the forward that keeps every composited
// fragment, which the recompute backward is measured against).
//
// Three launches over n counts: per-block sums (2048 counts per block), one
// workgroup scanning the block sums, and a pass writing every offset.
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__host__ __device__ inline int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

// Exclusive scan over the 256 threads of one value each; *total gets the sum.
__device__ uint32_t wg_exclusive_scan(uint32_t x, uint32_t* s_w, uint32_t& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        base += k < w ? s_w[k] : 0u;
        tot += s_w[k];
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void k_frag_block_sums(const uint32_t* __restrict__ count,
                                                                  int64_t n,
                                                                  uint32_t* __restrict__ sums)
{
    __shared__ uint32_t s_w[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) c += base + r < n ? count[base + r] : 0u;
    uint32_t tot;
    wg_exclusive_scan(c, s_w, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: sums[b] <- sum of sums[0..b), total[0] <- sum of all.
__global__ __launch_bounds__(kScanThreads) void k_frag_scan_sums(uint32_t* __restrict__ sums,
                                                                 int64_t nb,
                                                                 uint32_t* __restrict__ total)
{
    __shared__ uint32_t s_w[kScanThreads / 64];
    uint32_t running = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t x = b < nb ? sums[b] : 0u;
        uint32_t tot;
        const uint32_t pre = wg_exclusive_scan(x, s_w, tot);
        if (b < nb) sums[b] = running + pre;
        running += tot;
    }
    if (threadIdx.x == 0) total[0] = running;
}

__global__ __launch_bounds__(kScanThreads) void k_frag_offsets(const uint32_t* __restrict__ count,
                                                               int64_t n,
                                                               const uint32_t* __restrict__ sums,
                                                               uint32_t* __restrict__ offset)
{
    __shared__ uint32_t s_w[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t c[kScanItems], s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        c[r] = base + r < n ? count[base + r] : 0u;
        s += c[r];
    }
    uint32_t tot;
    uint32_t pre = wg_exclusive_scan(s, s_w, tot) + sums[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        if (base + r < n) offset[base + r] = pre;
        pre += c[r];
    }
}

}  // namespace

size_t fragment_scan_workspace_bytes(int64_t n)
{
    return sizeof(uint32_t) * (size_t)(scan_blocks(n > 0 ? n : 1) + 1);
}

void launch_fragment_offsets(const uint32_t* count, int64_t n, uint32_t* offset, uint32_t* total,
                             void* ws, hipStream_t stream)
{
    const int64_t nb = scan_blocks(n);
    uint32_t* sums = reinterpret_cast<uint32_t*>(ws);
    if (nb == 0) {
        launch_fill_u32(total, 1, 0u, stream);
        return;
    }
    hipLaunchKernelGGL(k_frag_block_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, count,
                       n, sums);
    hipLaunchKernelGGL(k_frag_scan_sums, dim3(1), dim3(kScanThreads), 0, stream, sums, nb, total);
    hipLaunchKernelGGL(k_frag_offsets, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, count, n,
                       (const uint32_t*)sums, offset);
}

}  // namespace ts
