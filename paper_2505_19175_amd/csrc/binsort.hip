// binsort.hip -- tile binning and (tile, depth) ordering on gfx950.
//
// The ordering the renderer needs is: instances grouped by tile, and inside a
// tile front to back by the depth key, ties by triangle index.  Sorting the
// 64-bit (tile, depth) keys of all M instances would take 6 radix passes over
// M.  Instead:
//   1. compact the visible triangles in index order            (N_v entries)
//   2. stable LSD radix sort of their depth keys, 4 x 8 bits   (N_v entries)
//   3. scan their tile counts in that order and emit one instance per tile,
//      so instances come out in (depth, index) order
//   4. stable LSD radix sort of the instances by tile id,
//      ceil(log2 tiles / 8) passes                               (M entries)
// A stable sort by tile of a sequence already ordered by (depth, index) is
// exactly the (tile, depth, index) order.
//
// Every pass is reduce-then-scan: per-block digit histograms, a scan of the
// histogram matrix, and a stable scatter whose in-block ranks come from
// wavefront ballots.  No kernel waits on another block, so nothing can spin.
// Element counts are read from device memory, so the whole chain can run
// without a host round trip (grids sized by upper bounds).
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kItems = 8;                    // keys per thread
constexpr int kChunk = kBlock * kItems;      // 2048 keys per block
constexpr int kRadix = 256;

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ static inline int64_t nblocks(int64_t n) { return (n + kChunk - 1) / kChunk; }

BinWorkspace carve_bin_workspace(void* base, int64_t N, uint64_t capacity)
{
    BinWorkspace w{};
    const int64_t nbN = nblocks(N > 0 ? N : 1);
    const int64_t nbC = nblocks(capacity > 0 ? (int64_t)capacity : 1);
    w.hist_stride = nbN > nbC ? nbN : nbC;
    char* p = reinterpret_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = p ? p + off : nullptr;
        off += align256(bytes);
        return reinterpret_cast<uint32_t*>(q);
    };
    const size_t n4 = 4 * (size_t)(N > 0 ? N : 1);
    const size_t c4 = 4 * (size_t)(capacity > 0 ? capacity : 1);
    w.blk = take(4 * (size_t)(w.hist_stride + 1));
    w.dk[0] = take(n4);
    w.dk[1] = take(n4);
    w.dv[0] = take(n4);
    w.dv[1] = take(n4);
    w.off = take(4);
    w.hist = take(4 * (size_t)kRadix * (size_t)w.hist_stride);
    w.dtot = take(4 * kRadix);
    w.tk[0] = take(c4);
    w.tk[1] = take(c4);
    w.tv[0] = take(c4);
    w.tv[1] = take(c4);
    w.tfin = take(c4);
    w.ctl = take(4 * 8);
    w.bytes = off;
    return w;
}

// ---------------------------------------------------------------------------
// Block-wide scan of one value per thread (256 threads).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t& total,
                                                         uint32_t* s_tmp)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < kBlock / 64; ++j) {
        const uint32_t t = s_tmp[j];
        wbase += j < w ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - x;
}

// ---------------------------------------------------------------------------
// 1. compaction of visible triangles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_count_visible(const uint32_t* __restrict__ ntiles,
                                                       int64_t N_host,
                                                       const uint32_t* __restrict__ d_n,
                                                       uint32_t* __restrict__ blk)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    if ((int64_t)blockIdx.x >= nblocks(N)) return;
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r;
        c += (i < N && ntiles[i] != 0u) ? 1u : 0u;
    }
    uint32_t tot;
    block_exclusive_scan(c, tot, s_tmp);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Exclusive scan in place of the per-block sums (one workgroup).  The number
// of blocks is nblocks(n) with n = *d_n (or n_host when d_n is null).  The
// total goes to total_out[0]; if cap_out is set, min(total, cap) goes to
// cap_out[0] and total > cap sets flag_out[0].
__global__ __launch_bounds__(256) void k_scan_blocks(uint32_t* __restrict__ blk,
                                                     const uint32_t* __restrict__ d_n,
                                                     int64_t n_host, uint32_t* total_out,
                                                     uint32_t* cap_out, uint64_t cap,
                                                     uint32_t* flag_out)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t n = d_n ? (int64_t)*d_n : n_host;
    const int64_t nb = nblocks(n);
    uint32_t running = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kBlock * 4) {
        uint32_t x[4], s = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = c0 + threadIdx.x * 4 + r;
            x[r] = j < nb ? blk[j] : 0u;
            s += x[r];
        }
        uint32_t tot;
        uint32_t pre = block_exclusive_scan(s, tot, s_tmp) + running;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = c0 + threadIdx.x * 4 + r;
            if (j < nb) blk[j] = pre;
            pre += x[r];
        }
        running += tot;
    }
    if (threadIdx.x == 0) {
        total_out[0] = running;
        if (cap_out) {
            cap_out[0] = (uint64_t)running > cap ? (uint32_t)cap : running;
            flag_out[0] = (uint64_t)running > cap ? 1u : 0u;
        }
    }
}

__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ ntiles,
                                                 const float* __restrict__ depth, int64_t N_host,
                                                 const uint32_t* __restrict__ d_n,
                                                 const uint32_t* __restrict__ blk,
                                                 uint32_t* __restrict__ dk,
                                                 uint32_t* __restrict__ dv)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    if ((int64_t)blockIdx.x >= nblocks(N)) return;
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
    uint32_t f[kItems], c = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r;
        f[r] = (i < N && ntiles[i] != 0u) ? 1u : 0u;
        c += f[r];
    }
    uint32_t tot;
    uint32_t pos = block_exclusive_scan(c, tot, s_tmp) + blk[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (f[r]) {
            const int64_t i = base + r;
            dk[pos] = __float_as_uint(depth[i]);   // positive floats order as unsigned ints
            dv[pos] = (uint32_t)i;
            ++pos;
        }
    }
}

// ---------------------------------------------------------------------------
// 2./4. stable LSD radix sort pass (8-bit digit at `shift`)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ d_n, int shift,
                                                    uint32_t* __restrict__ hist,
                                                    int64_t stride)
{
    __shared__ uint32_t h[kRadix];
    const int64_t n = *d_n;
    const int64_t b = blockIdx.x;
    if (b >= nblocks(n)) return;
    h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = b * kChunk + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * stride + b] = h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of that digit's row of block counts.
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* __restrict__ hist,
                                                    const uint32_t* __restrict__ d_n,
                                                    int64_t stride, uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t nb = nblocks(*d_n);
    uint32_t* row = hist + blockIdx.x * stride;
    uint32_t running = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kBlock * 4) {
        uint32_t x[4], s = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = c0 + threadIdx.x * 4 + r;
            x[r] = j < nb ? row[j] : 0u;
            s += x[r];
        }
        uint32_t tot;
        uint32_t pre = block_exclusive_scan(s, tot, s_tmp) + running;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = c0 + threadIdx.x * 4 + r;
            if (j < nb) row[j] = pre;
            pre += x[r];
        }
        running += tot;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = running;
}

// Stable scatter.  Keys of a block are read striped (key r*256 + tid), so the
// stable order inside the block is (round, wave, lane).  Each wave finds the
// lanes sharing its digit with 8 ballots; per (round, wave, digit) counts in
// LDS are scanned per digit to give every key its rank.
__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_n,
    int shift, const uint32_t* __restrict__ hist, int64_t stride,
    const uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint16_t s_cnt[kItems * 4][kRadix];
    __shared__ uint32_t s_tmp[4];
    const int64_t n = *d_n;
    const int64_t b = blockIdx.x;
    if (b >= nblocks(n)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

    uint32_t tot;
    const uint32_t dpre = block_exclusive_scan(dtot[tid], tot, s_tmp);
    s_base[tid] = dpre + hist[tid * stride + b];
#pragma unroll
    for (int s = 0; s < kItems * 4; ++s) s_cnt[s][tid] = 0;
    __syncthreads();

    uint32_t key[kItems], val[kItems], rank[kItems];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = b * kChunk + r * kBlock + tid;
        const bool ok = i < n;
        key[r] = ok ? kin[i] : 0u;
        val[r] = ok ? vin[i] : 0u;
        const uint32_t d = (key[r] >> shift) & 0xffu;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t bal = __ballot(set);
            m &= set ? bal : ~bal;
        }
        rank[r] = (uint32_t)__popcll(m & lt);
        if (ok && (m & lt) == 0ull) s_cnt[r * 4 + w][d] = (uint16_t)__popcll(m);
    }
    __syncthreads();
    {
        uint32_t run = 0;
#pragma unroll
        for (int s = 0; s < kItems * 4; ++s) {
            const uint32_t c = s_cnt[s][tid];
            s_cnt[s][tid] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = b * kChunk + r * kBlock + tid;
        if (i < n) {
            const uint32_t d = (key[r] >> shift) & 0xffu;
            const uint32_t pos = s_base[d] + s_cnt[r * 4 + w][d] + rank[r];
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

// ---------------------------------------------------------------------------
// 3. instances of the depth-sorted triangles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_count_instances(const uint32_t* __restrict__ ntiles,
                                                         const uint32_t* __restrict__ dv,
                                                         const uint32_t* __restrict__ d_nv,
                                                         uint32_t* __restrict__ blk)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t n = *d_nv;
    if ((int64_t)blockIdx.x >= nblocks(n)) return;
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t j = base + r;
        c += j < n ? ntiles[dv[j]] : 0u;
    }
    uint32_t tot;
    block_exclusive_scan(c, tot, s_tmp);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ ntiles,
                                              const short4* __restrict__ rect,
                                              const uint32_t* __restrict__ dv,
                                              const uint32_t* __restrict__ d_nv,
                                              const uint32_t* __restrict__ blk, int tiles_x,
                                              const ts_view* __restrict__ views, int64_t per_view,
                                              uint64_t capacity, uint32_t* __restrict__ tk,
                                              uint32_t* __restrict__ tv)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t n = *d_nv;
    if ((int64_t)blockIdx.x >= nblocks(n)) return;
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
    uint32_t cnt[kItems], tri[kItems], c = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t j = base + r;
        tri[r] = j < n ? dv[j] : 0u;
        cnt[r] = j < n ? ntiles[tri[r]] : 0u;
        c += cnt[r];
    }
    uint32_t tot;
    uint64_t pos = block_exclusive_scan(c, tot, s_tmp) + (uint64_t)blk[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (cnt[r] == 0u) continue;
        const short4 rc = rect[tri[r]];
        const int tx0 = rc.x / kTile, tx1 = rc.y / kTile;
        const int ty0 = rc.z / kTile, ty1 = rc.w / kTile;
        uint32_t toff = 0;
        int tw = tiles_x;
        if (views) {   // batched: entry = view * per_view + triangle
            const ts_view& V = views[tri[r] / (uint64_t)per_view];
            toff = V.tile_offset;
            tw = (int)V.tiles_x;
        }
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                if (pos < capacity) {
                    tk[pos] = toff + (uint32_t)(ty * tw + tx);
                    tv[pos] = tri[r];
                }
                ++pos;
            }
    }
}

// ---------------------------------------------------------------------------
// ranges and (optional) 64-bit keys
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = x;
}

// Batch descriptor as the kernels use it, clamped to the buffers' sizes:
// out[0] = views, out[1] = tiles, out[2] = views * per_view entries.
__global__ void k_batch_ctl(const uint32_t* __restrict__ ctl_in, uint32_t max_views,
                            uint32_t max_tiles, int64_t per_view, uint32_t* __restrict__ ctl_out)
{
    if (threadIdx.x == 0) {
        const uint32_t nv = min(ctl_in[0], max_views);
        ctl_out[0] = nv;
        ctl_out[1] = min(ctl_in[1], max_tiles);
        ctl_out[2] = (uint32_t)((int64_t)nv * per_view);
    }
}

void launch_batch_ctl(const uint32_t* ctl_in, uint32_t max_views, uint32_t max_tiles,
                      int64_t per_view, uint32_t* ctl_out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_ctl, dim3(1), dim3(64), 0, stream, ctl_in, max_views, max_tiles,
                       per_view, ctl_out);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t x, hipStream_t stream)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, x);
}

// Tiles by decreasing list length (counting sort on the length, lengths of
// 2047 and more share the first bucket; order inside a bucket is arbitrary).
// Rasterizing the longest tiles first keeps them out of the tail of the
// launch.  One workgroup; ctl (optional) holds the number of tiles.
constexpr int kLenBuckets = 2048;

__global__ __launch_bounds__(256) void k_tile_order(const uint32_t* __restrict__ ranges,
                                                    int n_host, const uint32_t* __restrict__ d_n,
                                                    uint32_t* __restrict__ order)
{
    __shared__ uint32_t h[kLenBuckets];
    __shared__ uint32_t s_tmp[4];
    const int n = d_n ? (int)min(*d_n, (uint32_t)n_host) : n_host;
    for (int b = threadIdx.x; b < kLenBuckets; b += kBlock) h[b] = 0u;
    __syncthreads();
    auto key = [&](int t) {
        const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        return (kLenBuckets - 1) - (int)min(len, (uint32_t)(kLenBuckets - 1));
    };
    for (int t = threadIdx.x; t < n; t += kBlock) atomicAdd(&h[key(t)], 1u);
    __syncthreads();
    constexpr int per = kLenBuckets / kBlock;
    uint32_t loc[per], s = 0;
#pragma unroll
    for (int r = 0; r < per; ++r) {
        loc[r] = h[threadIdx.x * per + r];
        s += loc[r];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, tot, s_tmp);
#pragma unroll
    for (int r = 0; r < per; ++r) {
        h[threadIdx.x * per + r] = pre;
        pre += loc[r];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += kBlock) order[atomicAdd(&h[key(t)], 1u)] = (uint32_t)t;
}

void launch_tile_order(const uint32_t* ranges, int num_tiles, const uint32_t* d_tiles,
                       uint32_t* order, hipStream_t stream)
{
    if (order && num_tiles > 0)
        hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kBlock), 0, stream, ranges, num_tiles,
                           d_tiles, order);
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tfin,
                                                const uint32_t* __restrict__ vals,
                                                const float* __restrict__ depth,
                                                const uint32_t* __restrict__ d_m,
                                                uint32_t* __restrict__ ranges,
                                                uint64_t* __restrict__ keys)
{
    const int64_t m = *d_m;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const uint32_t t = tfin[p];
    if (p == 0 || tfin[p - 1] != t) ranges[2 * t] = (uint32_t)p;
    if (p == m - 1 || tfin[p + 1] != t) ranges[2 * t + 1] = (uint32_t)(p + 1);
    if (keys) keys[p] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(depth[vals[p]]);
}

// ---------------------------------------------------------------------------

static hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                             uint32_t* kfin, uint32_t* vfin, const uint32_t* d_n,
                             int64_t n_max, int bits, const BinWorkspace& ws,
                             hipStream_t stream)
{
    const int passes = (bits + 7) / 8;
    const int64_t nb = nblocks(n_max > 0 ? n_max : 1);
    uint32_t* ks[2] = {k0, k1};
    uint32_t* vs[2] = {v0, v1};
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const bool last = p == passes - 1;
        uint32_t* ko = last ? kfin : ks[src ^ 1];
        uint32_t* vo = last ? vfin : vs[src ^ 1];
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, stream, ks[src], d_n,
                           shift, ws.hist, ws.hist_stride);
        hipLaunchKernelGGL(k_radix_scan, dim3(kRadix), dim3(kBlock), 0, stream, ws.hist, d_n,
                           ws.hist_stride, ws.dtot);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, stream, ks[src],
                           vs[src], ko, vo, d_n, shift, ws.hist, ws.hist_stride, ws.dtot);
        src ^= 1;
    }
    return hipGetLastError();
}

static int bits_for(int n)
{
    int b = 0;
    while ((1 << b) < n) ++b;
    return b > 0 ? b : 1;
}

hipError_t run_bin_sort(const uint32_t* ntiles, const float* depth, const int16_t* rect,
                        int64_t N, const uint32_t* d_n, const ts_view* views, int64_t per_view,
                        int tiles_x, int num_tiles, const BinWorkspace& ws, const ts_bins& out,
                        uint32_t* h_count, bool* overflow, hipStream_t stream,
                        const uint32_t* d_tiles)
{
    *overflow = false;
    const int64_t nbN = nblocks(N);
    uint32_t* d_M = out.d_count;        // [0] M
    uint32_t* d_Nv = out.d_count + 1;   // [1] N_v
    uint32_t* d_ovf = out.d_count + 2;  // [2] overflow
    uint32_t* d_sortn = ws.ctl;         // min(M, capacity)

    launch_fill_u32(out.ranges, 2 * (int64_t)num_tiles, 0u, stream);
    // 1. compaction (N, or *d_n entries when given)
    hipLaunchKernelGGL(k_count_visible, dim3((unsigned)nbN), dim3(kBlock), 0, stream, ntiles, N,
                       d_n, ws.blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, stream, ws.blk, d_n, N, d_Nv,
                       (uint32_t*)nullptr, (uint64_t)0, (uint32_t*)nullptr);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nbN), dim3(kBlock), 0, stream, ntiles, depth, N,
                       d_n, ws.blk, ws.dk[0], ws.dv[0]);
    // 2. depth order of the visible triangles (stable: index order kept on ties)
    hipError_t err = radix_sort(ws.dk[0], ws.dv[0], ws.dk[1], ws.dv[1], ws.dk[0], ws.dv[0], d_Nv,
                                N, 32, ws, stream);
    if (err != hipSuccess) return err;
    // 3. instance offsets and emission in depth order
    hipLaunchKernelGGL(k_count_instances, dim3((unsigned)nbN), dim3(kBlock), 0, stream, ntiles,
                       ws.dv[0], d_Nv, ws.blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, stream, ws.blk, d_Nv, (int64_t)0,
                       d_M, d_sortn, out.capacity, d_ovf);
    int64_t m_max = (int64_t)out.capacity;
    if (h_count) {
        err = hipMemcpyAsync(h_count, out.d_count, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                             stream);
        if (err != hipSuccess) return err;
        err = hipStreamSynchronize(stream);
        if (err != hipSuccess) return err;
        if ((uint64_t)h_count[0] > out.capacity) {
            // ranges are all empty here; keep the order valid for any raster
            // launched before the caller grows the list
            *overflow = true;
            launch_tile_order(out.ranges, num_tiles, d_tiles, out.order, stream);
            return hipGetLastError();
        }
        m_max = h_count[0];
    }
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nbN), dim3(kBlock), 0, stream, ntiles,
                       reinterpret_cast<const short4*>(rect), ws.dv[0], d_Nv, ws.blk, tiles_x,
                       views, per_view, out.capacity, ws.tk[0], ws.tv[0]);
    // 4. stable sort by tile
    err = radix_sort(ws.tk[0], ws.tv[0], ws.tk[1], ws.tv[1], ws.tfin, out.vals, d_sortn, m_max,
                     bits_for(num_tiles), ws, stream);
    if (err != hipSuccess) return err;
    if (m_max > 0)
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((m_max + 255) / 256)), dim3(256), 0, stream,
                           ws.tfin, out.vals, depth, d_sortn, out.ranges, out.keys);
    launch_tile_order(out.ranges, num_tiles, d_tiles, out.order, stream);
    return hipGetLastError();
}

}  // namespace ts
