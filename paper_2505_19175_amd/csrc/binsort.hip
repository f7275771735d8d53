// binsort.hip -- tile binning and (tile, depth) ordering on gfx950.
//
// The ordering the renderer needs is: instances grouped by tile, and inside a
// tile front to back by the depth key, ties by triangle index.  Sorting the
// 64-bit (tile, depth) keys of all M instances would take 6 radix passes over
// M.  Instead the instances are first grouped by tile, then each tile's run
// is put in depth order.  Grouping, when the tile counters fit in LDS (up to
// kGroupTiles tiles) and the huge tiles are not sorted segment-wise:
//   1'. G groups of consecutive triangles count their instances per tile in
//       LDS (a G x tiles matrix), a column scan gives each group its offset
//       inside each tile, one workgroup scans the tile totals into the ranges
//       and the longest-first tile order, and the groups place every instance
//       at tile start + group offset + an LDS cursor (four launches, no pass
//       over the instance list)
// Otherwise (more tiles, or the segmented sort of huge tiles, which needs the
// runs in index order):
//   1. count the tiles of every triangle, in index order, and scan the counts
//   2. emit one instance per (triangle, tile) in index order
//   3. stable LSD radix sort of the instances by tile id,
//      ceil(log2 tiles / 8) passes over M with the bits split evenly between
//      them; inside a tile the triangles are still in index order
// Then:
//   4. each tile's entries are put in (depth key, index) order: up to 128
//      entries by one wave, a bitonic network over 64-bit (depth, index)
//      keys held in registers; up to 4096 by four waves (a quarter each) and
//      a merge in LDS; beyond, a stable radix sort by depth of the run in
//      index order (one workgroup with global ping-pong buffers, which first
//      sorts by index a run that step 1' left in group order, or the
//      segmented sort below), skipping the 8-bit digits equal over the tile
// The keys of the networks are unique, and a stable sort by depth of a list
// in index order is the (depth, index) order, so either way the result is
// exactly the (tile, depth, index) order.
//
// Every global pass of steps 1-3 is reduce-then-scan: per-block digit
// histograms, a scan of the histogram matrix, and a stable scatter whose
// in-block ranks come from wavefront ballots and the group leaders' returned
// LDS counts, staged in LDS so the block writes runs of consecutive
// addresses.  No kernel waits on another block, so nothing can spin.
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

BinWorkspace carve_bin_workspace(void* base, int64_t N, uint64_t capacity, int64_t num_tiles)
{
    BinWorkspace w{};
    const int64_t nbN = nblocks(N > 0 ? N : 1);
    const int64_t nbC = nblocks(capacity > 0 ? (int64_t)capacity : 1);
    // the segmented sort's chunks: at most one partial chunk per tile more
    w.hist_stride = nbC + (num_tiles > 0 ? num_tiles : 1);
    char* p = reinterpret_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = p ? p + off : nullptr;
        off += align256(bytes);
        return reinterpret_cast<uint32_t*>(q);
    };
    const size_t c4 = 4 * (size_t)(capacity > 0 ? capacity : 1);
    w.blk = take(4 * (size_t)(nbN + 1));
    w.blk_vis = take(4 * (size_t)(nbN + 1));
    w.hist = take(4 * (size_t)kRadix * (size_t)w.hist_stride);
    w.dtot = take(4 * kRadix);
    w.tk[0] = take(c4);
    w.tk[1] = take(c4);
    w.tv[0] = take(c4);
    w.tv[1] = take(c4);
    w.tfin = take(c4);
    w.torder = take(4 * (size_t)(num_tiles > 0 ? num_tiles : 1));
    w.hl = take(4 * (size_t)(num_tiles > 0 ? num_tiles : 1));
    w.cst = take(4 * (size_t)(num_tiles + 2));
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
// 1. tile counts in index order
// ---------------------------------------------------------------------------
// Per block of kChunk entries: the number of instances and of visible
// entries.  The grid also clears the n_ranges words of the tile ranges.
__global__ __launch_bounds__(256) void k_count(const uint32_t* __restrict__ ntiles,
                                               int64_t N_host, const uint32_t* __restrict__ d_n,
                                               uint32_t* __restrict__ blk,
                                               uint32_t* __restrict__ blk_vis,
                                               uint32_t* __restrict__ ranges, int64_t n_ranges)
{
    __shared__ uint32_t s_tmp[4];
    for (int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x; f < n_ranges;
         f += (int64_t)gridDim.x * kBlock)
        ranges[f] = 0u;
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    if ((int64_t)blockIdx.x >= nblocks(N)) return;
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
    uint32_t c = 0, v = 0;
    if (base + kItems <= N && (reinterpret_cast<uintptr_t>(ntiles + base) & 15u) == 0u) {
        const uint4* p4 = reinterpret_cast<const uint4*>(ntiles + base);
#pragma unroll
        for (int r = 0; r < kItems / 4; ++r) {
            const uint4 q = p4[r];
            c += q.x + q.y + q.z + q.w;
            v += (q.x != 0u) + (q.y != 0u) + (q.z != 0u) + (q.w != 0u);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t i = base + r;
            const uint32_t n = i < N ? ntiles[i] : 0u;
            c += n;
            v += n != 0u ? 1u : 0u;
        }
    }
    uint32_t tot, tot_vis;
    block_exclusive_scan(c, tot, s_tmp);
    block_exclusive_scan(v, tot_vis, s_tmp);
    if (threadIdx.x == 0) {
        blk[blockIdx.x] = tot;
        blk_vis[blockIdx.x] = tot_vis;
    }
}

// ---------------------------------------------------------------------------
// 2. instances in index order
// ---------------------------------------------------------------------------
// The block's instances fill one contiguous range of the list, written slot
// by slot by consecutive lanes (coalesced): slot q finds its entry by a
// binary search over the per-thread prefix counts, then a walk over that
// thread's kItems entries, and its tile from the entry's tile rectangle.
// The block's first output slot is the sum of the counts of the blocks before
// it (k_count's per-block totals, summed here by each block: no separate scan
// launch); the last block also writes the totals: M, min(M, capacity) for the
// sort, the overflow flag and N_v.
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ ntiles,
                                              const short4* __restrict__ rect, int64_t N_host,
                                              const uint32_t* __restrict__ d_n,
                                              const uint32_t* __restrict__ blk,
                                              const uint32_t* __restrict__ blk_vis, int tiles_x,
                                              const ts_view* __restrict__ views, int64_t per_view,
                                              uint64_t capacity, uint32_t* __restrict__ tk,
                                              uint32_t* __restrict__ tv, uint32_t* __restrict__ d_M,
                                              uint32_t* __restrict__ d_sortn,
                                              uint32_t* __restrict__ d_ovf,
                                              uint32_t* __restrict__ d_Nv)
{
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_pre[kBlock];         // instances before each thread's entries
    __shared__ uint32_t s_cnt[kChunk];         // tiles of entry tid * kItems + r at r * kBlock + tid
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    const int64_t nb = nblocks(N);
    if (nb == 0) {   // nothing to emit: the totals are zero
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *d_M = 0u; *d_sortn = 0u; *d_ovf = 0u; *d_Nv = 0u;
        }
        return;
    }
    if ((int64_t)blockIdx.x >= nb) return;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const bool last_block = (int64_t)blockIdx.x == nb - 1;
    uint32_t before = 0, vis = 0;
    for (int64_t b = tid; b < (int64_t)blockIdx.x; b += kBlock) before += blk[b];
    if (last_block)
        for (int64_t b = tid; b < nb; b += kBlock) vis += blk_vis[b];
    uint32_t c = 0;
    const int64_t e0 = base + tid * kItems;
    if (e0 + kItems <= N && (reinterpret_cast<uintptr_t>(ntiles + e0) & 15u) == 0u) {
        const uint4* p4 = reinterpret_cast<const uint4*>(ntiles + e0);
#pragma unroll
        for (int r = 0; r < kItems / 4; ++r) {
            const uint4 q = p4[r];
            s_cnt[(4 * r + 0) * kBlock + tid] = q.x;
            s_cnt[(4 * r + 1) * kBlock + tid] = q.y;
            s_cnt[(4 * r + 2) * kBlock + tid] = q.z;
            s_cnt[(4 * r + 3) * kBlock + tid] = q.w;
            c += q.x + q.y + q.z + q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t i = e0 + r;
            const uint32_t n = i < N ? ntiles[i] : 0u;
            s_cnt[r * kBlock + tid] = n;
            c += n;
        }
    }
    uint32_t tot, out0_32, vis_tot;
    s_pre[tid] = block_exclusive_scan(c, tot, s_tmp);
    block_exclusive_scan(before, out0_32, s_tmp);
    if (last_block) {
        block_exclusive_scan(vis, vis_tot, s_tmp);
        if (tid == 0) {
            const uint64_t M = (uint64_t)out0_32 + tot;
            *d_M = (uint32_t)M;
            *d_sortn = M > capacity ? (uint32_t)capacity : (uint32_t)M;
            *d_ovf = M > capacity ? 1u : 0u;
            *d_Nv = vis_tot;
        }
    }
    __syncthreads();
    const uint64_t out0 = (uint64_t)out0_32;
    for (uint32_t q = tid; q < tot; q += kBlock) {
        if (out0 + q >= capacity) break;
        int t = 0;   // last thread whose first instance is at or before q
#pragma unroll
        for (int step = kBlock / 2; step > 0; step >>= 1)
            if (s_pre[t + step] <= q) t += step;
        uint32_t k = q - s_pre[t];
        int r = 0;
        while (k >= s_cnt[r * kBlock + t]) {   // ends within the thread's entries
            k -= s_cnt[r * kBlock + t];
            ++r;
        }
        const uint32_t e = (uint32_t)(base + t * kItems + r);
        const short4 rc = rect[e];
        const int tx0 = rc.x / kTile, nx = rc.y / kTile - tx0 + 1, ty0 = rc.z / kTile;
        uint32_t toff = 0;
        int tw = tiles_x;
        if (views) {   // batched: entry = view * per_view + triangle
            const ts_view& V = views[e / (uint64_t)per_view];
            toff = V.tile_offset;
            tw = (int)V.tiles_x;
        }
        const int dy = (int)(k / (uint32_t)nx), dx = (int)(k - (uint32_t)(dy * nx));
        tk[out0 + q] = toff + (uint32_t)((ty0 + dy) * tw + tx0 + dx);
        tv[out0 + q] = e;
    }
}

// ---------------------------------------------------------------------------
// 3. stable LSD radix sort pass (digit of `dbits` <= 8 bits at `shift`)
// ---------------------------------------------------------------------------
// The passes split the key's bits evenly (12 bits of tile id: two 6-bit
// digits), so a block's keys fall into fewer, longer runs.
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ d_n, int shift,
                                                    int dbits, uint32_t* __restrict__ hist,
                                                    int64_t stride)
{
    __shared__ uint32_t h[kRadix];
    const int64_t n = *d_n;
    const int64_t b = blockIdx.x;
    if (b >= nblocks(n)) return;
    const uint32_t mask = (1u << dbits) - 1u;
    h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = b * kChunk + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= mask) hist[threadIdx.x * stride + b] = h[threadIdx.x];
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

// Stable scatter.  Wave w of a block reads keys w * 512 + r * 64 + lane of the
// block's 2048 (round r), so the stable order inside the block is (wave,
// round, lane).  In each round the lanes sharing a digit are found with dbits
// ballots; the group's leader adds the group size to its wave's count of the
// digit and gets back the count before it (the wave's earlier rounds: a
// wave's LDS operations take effect in program order).  The block's keys are
// then placed in LDS in their sorted order and written out by consecutive
// lanes, so a store instruction covers a few runs of consecutive addresses
// instead of up to 64 scattered words.
__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_n,
    int shift, int dbits, const uint32_t* __restrict__ hist, int64_t stride,
    const uint32_t* __restrict__ dtot)
{
    constexpr int kWaveKeys = kChunk / (kBlock / 64);   // 512 keys per wave
    __shared__ uint32_t s_off[kRadix];   // output position of the block's k-th key of digit d: s_off[d] + k
    __shared__ uint32_t s_lst[kRadix];   // first LDS slot of digit d
    __shared__ uint32_t s_cnt[kBlock / 64][kRadix];   // per wave and digit: count, then the waves before
    __shared__ uint32_t s_key[kChunk];
    __shared__ uint32_t s_val[kChunk];
    __shared__ uint32_t s_tmp[4];
    const int64_t n = *d_n;
    const int64_t b = blockIdx.x;
    if (b >= nblocks(n)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t mask = (1u << dbits) - 1u;
    const int nloc = (int)min<int64_t>(kChunk, n - b * kChunk);

    uint32_t tot;
    const bool dig = (uint32_t)tid <= mask;
    const uint32_t dpre = block_exclusive_scan(dig ? dtot[tid] : 0u, tot, s_tmp);
    const uint32_t gbase = dig ? dpre + hist[tid * stride + b] : 0u;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) s_cnt[q][tid] = 0u;
    __syncthreads();

    uint32_t key[kItems], val[kItems], within[kItems];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int j = w * kWaveKeys + r * 64 + lane;
        const bool ok = j < nloc;
        key[r] = ok ? kin[b * kChunk + j] : 0u;
        val[r] = ok ? vin[b * kChunk + j] : 0u;
        const uint32_t d = (key[r] >> shift) & mask;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            if (bit < dbits) {   // the same for the whole block
                const bool set = (d >> bit) & 1u;
                const uint64_t bal = __ballot(set);
                m &= set ? bal : ~bal;
            }
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t lead = m != 0ull ? (uint32_t)__builtin_ctzll(m) : (uint32_t)lane;
        uint32_t before = 0u;
        if (ok && rank == 0u) before = atomicAdd(&s_cnt[w][d], (uint32_t)__popcll(m));
        within[r] = (uint32_t)__shfl((int)before, (int)lead, 64) + rank;
    }
    __syncthreads();
    // per digit: the counts of the waves before each wave, and the block's count
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
        const uint32_t c = s_cnt[q][tid];
        s_cnt[q][tid] = run;
        run += c;
    }
    uint32_t btot;
    const uint32_t lstart = block_exclusive_scan(run, btot, s_tmp);   // barriers inside
    s_lst[tid] = lstart;
    s_off[tid] = gbase - lstart;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (w * kWaveKeys + r * 64 + lane < nloc) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t q = s_lst[d] + s_cnt[w][d] + within[r];
            s_key[q] = key[r];
            s_val[q] = val[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int j = r * kBlock + tid;
        if (j < nloc) {
            const uint32_t k = s_key[j];
            const uint32_t pos = s_off[(k >> shift) & mask] + (uint32_t)j;
            kout[pos] = k;
            vout[pos] = s_val[j];
        }
    }
}

// ---------------------------------------------------------------------------
// fills, batch descriptor, tile order, ranges
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

// n_long (optional) receives the number of tiles longer than kWaveSortMax:
// they lead the order, since kWaveSortMax < kLenBuckets - 1.
constexpr int kWaveMax = 1024;   // longest list one wave's register network holds
// Longer lists get a whole workgroup (four quarter sorts and a merge): the
// quarters' shorter compare-exchange chains finish sooner than one wave's.
constexpr int kWaveSortMax = 128;
static_assert(kWaveSortMax <= kWaveMax && kWaveSortMax < kLenBuckets - 1,
              "long tiles must lead the order");

constexpr int kOrderThreads = 1024;

constexpr int kHugeLen = 4 * kWaveMax;   // longest list one workgroup sorts in LDS

// The order of tiles 0 .. n-1 by one workgroup of kOrderThreads; len_of(t)
// gives a tile's list length.
struct OrderSmem {
    uint32_t h[kLenBuckets];
    uint32_t w[kOrderThreads / 64];
    uint32_t nlong, nhuge;
};

template <class Len>
__device__ void order_tiles(int n, Len len_of, uint32_t* __restrict__ order,
                            uint32_t* __restrict__ n_long, uint32_t* __restrict__ n_huge,
                            OrderSmem& sm)
{
    uint32_t* h = sm.h;
    uint32_t* s_w = sm.w;
    uint32_t& s_long = sm.nlong;
    uint32_t& s_huge = sm.nhuge;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int b = tid; b < kLenBuckets; b += kOrderThreads) h[b] = 0u;
    if (tid == 0) {
        s_long = 0u;
        s_huge = 0u;
    }
    __syncthreads();
    auto key = [&](int t) {
        return (kLenBuckets - 1) - (int)min(len_of(t), (uint32_t)(kLenBuckets - 1));
    };
    for (int t = tid; t < n; t += kOrderThreads) {
        atomicAdd(&h[key(t)], 1u);
        if (len_of(t) > (uint32_t)kWaveSortMax) atomicAdd(&s_long, 1u);
        if (len_of(t) > (uint32_t)kHugeLen) atomicAdd(&s_huge, 1u);
    }
    __syncthreads();
    if (n_long && tid == 0) n_long[0] = s_long;
    if (n_huge && tid == 0) n_huge[0] = s_huge;
    // exclusive scan of the bucket counts, two consecutive buckets per thread
    static_assert(kLenBuckets == 2 * kOrderThreads, "two buckets per thread");
    const uint32_t a0 = h[2 * tid], a1 = h[2 * tid + 1], sum = a0 + a1;
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = inc - sum;
    for (int j = 0; j < w; ++j) pre += s_w[j];
    h[2 * tid] = pre;
    h[2 * tid + 1] = pre + a0;
    __syncthreads();
    for (int t = tid; t < n; t += kOrderThreads) order[atomicAdd(&h[key(t)], 1u)] = (uint32_t)t;
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(
    const uint32_t* __restrict__ ranges, int n_host, const uint32_t* __restrict__ d_n,
    uint32_t* __restrict__ order, uint32_t* __restrict__ n_long, uint32_t* __restrict__ n_huge)
{
    __shared__ OrderSmem sm;
    const int n = d_n ? (int)min(*d_n, (uint32_t)n_host) : n_host;
    order_tiles(
        n, [&](int t) { return ranges[2 * t + 1] - ranges[2 * t]; }, order, n_long, n_huge, sm);
}

void launch_tile_order(const uint32_t* ranges, int num_tiles, const uint32_t* d_tiles,
                       uint32_t* order, hipStream_t stream, uint32_t* n_long, uint32_t* n_huge)
{
    if (order && num_tiles > 0)
        hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, stream, ranges,
                           num_tiles, d_tiles, order, n_long, n_huge);
}


__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tfin,
                                                const uint32_t* __restrict__ d_m,
                                                uint32_t* __restrict__ ranges)
{
    const int64_t m = *d_m;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const uint32_t t = tfin[p];
    if (p == 0 || tfin[p - 1] != t) ranges[2 * t] = (uint32_t)p;
    if (p == m - 1 || tfin[p + 1] != t) ranges[2 * t + 1] = (uint32_t)(p + 1);
}

// ---------------------------------------------------------------------------
// 1'. grouping by group tile counts (up to kGroupTiles tiles)
// ---------------------------------------------------------------------------
// When the tile counters fit in LDS, steps 1-3 become four launches with no
// pass over the instance list: G groups of consecutive entries count their
// instances per tile in LDS (G x tiles matrix), a column scan turns the matrix
// into each group's offset inside each tile, one workgroup scans the tile
// totals into the ranges and the longest-first order, and the groups walk
// their entries again and place every instance at its tile's start + the
// group's offset + an LDS cursor.  Inside a tile the instances are then in
// group order but not in index order inside a group; the per-tile sort orders
// by the unique (depth, index) key anyway (the workgroup sort of the huge
// tiles sorts by index first).
constexpr int kGroupThreads = 1024;
constexpr int kMaxGroups = 256;
constexpr int kGroupEntries = 4096;   // fewest entries per group
constexpr int kGroupTiles = 12288;    // tile counters in LDS (48 KB)

constexpr int kGroupRun = 8;   // consecutive entries a thread loads at once

// The group a workgroup takes.  Workgroups are dealt to the eight XCDs in
// turn, so consecutive groups go to one XCD: they write neighbouring slots of
// every tile, and fewer cache lines are written in part by several XCDs'
// caches.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_group(int G)
{
    const int b = blockIdx.x;
    return (G % kXcds) == 0 ? (b % kXcds) * (G / kXcds) + b / kXcds : b;
}

// Entries [e0, e1) of group g: ceil(n / G), rounded up to whole runs.
__device__ __forceinline__ void group_span(int64_t n, int G, int g, int64_t& e0, int64_t& e1)
{
    int64_t per = (n + G - 1) / G;
    per = (per + kGroupRun - 1) / kGroupRun * kGroupRun;
    e0 = min(n, (int64_t)g * per);
    e1 = min(n, e0 + per);
}

// Tile counts and rectangles (x0, x1, y0, y1 as two words) of entries
// e .. e + kGroupRun - 1; counts at or past e1 read as zero.  Whole aligned
// runs use 16-byte loads, all issued before any is used.
__device__ __forceinline__ void load_run(const uint32_t* __restrict__ ntiles,
                                         const uint2* __restrict__ rect, int64_t e, int64_t e1,
                                         uint32_t (&n)[kGroupRun], uint2 (&rb)[kGroupRun])
{
    if (e + kGroupRun <= e1 && (reinterpret_cast<uintptr_t>(ntiles + e) & 15u) == 0u &&
        (reinterpret_cast<uintptr_t>(rect + e) & 15u) == 0u) {
        const uint4* pn = reinterpret_cast<const uint4*>(ntiles + e);
        const uint4* pr = reinterpret_cast<const uint4*>(rect + e);
        uint4 a[2], b[kGroupRun / 2];
#pragma unroll
        for (int r = 0; r < 2; ++r) a[r] = pn[r];
#pragma unroll
        for (int r = 0; r < kGroupRun / 2; ++r) b[r] = pr[r];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            n[4 * r + 0] = a[r].x;
            n[4 * r + 1] = a[r].y;
            n[4 * r + 2] = a[r].z;
            n[4 * r + 3] = a[r].w;
        }
#pragma unroll
        for (int r = 0; r < kGroupRun / 2; ++r) {
            rb[2 * r] = make_uint2(b[r].x, b[r].y);
            rb[2 * r + 1] = make_uint2(b[r].z, b[r].w);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kGroupRun; ++r) {
            n[r] = e + r < e1 ? ntiles[e + r] : 0u;
            rb[r] = n[r] != 0u ? rect[e + r] : make_uint2(0u, 0u);
        }
    }
}

// The first tile of entry e's rectangle, the rectangle's width in tiles and
// the tile row pitch.
struct TileWalk {
    uint32_t first;
    int nx, tw;
};

__device__ __forceinline__ TileWalk tile_walk(uint32_t e, uint2 rb, int tiles_x,
                                              const ts_view* __restrict__ views, int64_t per_view)
{
    const int x0 = (int16_t)(rb.x & 0xffffu), x1 = (int16_t)(rb.x >> 16);
    const int y0 = (int16_t)(rb.y & 0xffffu);
    const int tx0 = x0 / kTile, nx = x1 / kTile - tx0 + 1, ty0 = y0 / kTile;
    uint32_t toff = 0;
    int tw = tiles_x;
    if (views) {   // batched: entry = view * per_view + triangle
        const ts_view& V = views[e / (uint64_t)per_view];
        toff = V.tile_offset;
        tw = (int)V.tiles_x;
    }
    return {toff + (uint32_t)(ty0 * tw + tx0), nx, tw};
}

// Calls f(tile) for the n tiles of a rectangle, row by row.
template <class F>
__device__ __forceinline__ void for_tiles(const TileWalk& tw, uint32_t n, F f)
{
    uint32_t row = tw.first;
    int dx = 0;
    for (uint32_t k = 0; k < n; ++k) {
        f(row + (uint32_t)dx);
        if (++dx == tw.nx) {
            dx = 0;
            row += (uint32_t)tw.tw;
        }
    }
}

// Calls f(tile, entry) for every instance of the run's entries e .. e + 7:
// entries of up to kLaneTiles tiles by their own lane, larger ones (a
// triangle can cover hundreds of tiles) one at a time by all active lanes of
// the wave, so no lane walks a long rectangle alone.
constexpr uint32_t kLaneTiles = 8;

template <class F>
__device__ __forceinline__ void for_run_tiles(int64_t e, const uint32_t (&n)[kGroupRun],
                                              const uint2 (&rb)[kGroupRun], int tiles_x,
                                              const ts_view* __restrict__ views, int64_t per_view,
                                              F f)
{
#pragma unroll
    for (int r = 0; r < kGroupRun; ++r) {
        if (n[r] != 0u && n[r] <= kLaneTiles) {
            const uint32_t id = (uint32_t)(e + r);
            for_tiles(tile_walk(id, rb[r], tiles_x, views, per_view), n[r],
                      [&](uint32_t t) { f(t, id); });
        }
    }
    const uint64_t act = __ballot(1);
    const uint32_t nact = (uint32_t)__popcll(act);
    const int lane = threadIdx.x & 63;
    const uint32_t rank = (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
#pragma unroll
    for (int r = 0; r < kGroupRun; ++r) {
        uint64_t want = __ballot(n[r] > kLaneTiles);
        while (want != 0ull) {   // the same for all active lanes
            const int src = (int)__builtin_ctzll(want);
            want &= want - 1ull;
            const uint32_t ns = (uint32_t)__shfl((int)n[r], src, 64);
            const uint32_t id = (uint32_t)__shfl((int)(uint32_t)(e + r), src, 64);
            const uint2 rs = make_uint2((uint32_t)__shfl((int)rb[r].x, src, 64),
                                        (uint32_t)__shfl((int)rb[r].y, src, 64));
            const TileWalk tw = tile_walk(id, rs, tiles_x, views, per_view);
            for (uint32_t k = rank; k < ns; k += nact) {
                const uint32_t dy = k / (uint32_t)tw.nx, dx = k - dy * (uint32_t)tw.nx;
                f(tw.first + dy * (uint32_t)tw.tw + dx, id);
            }
        }
    }
}

// Per group: instances per tile (row g of hist, T wide), and the group's
// instance and visible-entry totals in grp[g], grp[G + g].
__global__ __launch_bounds__(kGroupThreads) void k_group_count(
    const uint32_t* __restrict__ ntiles, const uint2* __restrict__ rect, int64_t N_host,
    const uint32_t* __restrict__ d_n, int tiles_x, const ts_view* __restrict__ views,
    int64_t per_view, int T, int G, uint32_t* __restrict__ hist, uint32_t* __restrict__ grp)
{
    extern __shared__ uint32_t s_h[];   // [T]
    __shared__ uint32_t s_tmp[kGroupThreads / 64][2];
    const int tid = threadIdx.x, g = xcd_group(G);
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    int64_t e0, e1;
    group_span(N, G, g, e0, e1);
    for (int t = tid; t < T; t += kGroupThreads) s_h[t] = 0u;
    __syncthreads();
    uint32_t m = 0, v = 0;
    for (int64_t e = e0 + (int64_t)tid * kGroupRun; e < e1;
         e += (int64_t)kGroupThreads * kGroupRun) {
        uint32_t n[kGroupRun];
        uint2 rb[kGroupRun];
        load_run(ntiles, rect, e, e1, n, rb);
#pragma unroll
        for (int r = 0; r < kGroupRun; ++r) {
            m += n[r];
            v += n[r] != 0u ? 1u : 0u;
        }
        for_run_tiles(e, n, rb, tiles_x, views, per_view, [&](uint32_t t, uint32_t) {
            if (t < (uint32_t)T) atomicAdd(&s_h[t], 1u);
        });
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        m += __shfl_xor(m, d, 64);
        v += __shfl_xor(v, d, 64);
    }
    if ((tid & 63) == 0) {
        s_tmp[tid >> 6][0] = m;
        s_tmp[tid >> 6][1] = v;
    }
    __syncthreads();
    uint32_t* row = hist + (int64_t)g * T;
    for (int t = tid; t < T; t += kGroupThreads) row[t] = s_h[t];
    if (tid < 2) {
        uint32_t x = 0;
        for (int j = 0; j < kGroupThreads / 64; ++j) x += s_tmp[j][tid];
        grp[tid * G + g] = x;
    }
}

// Column scan: hist[g][t] becomes the instances of tile t in groups before g;
// tot[t] the tile's total.  64 tiles per workgroup; each of its 16 waves holds
// a slice of up to 16 groups in registers.
constexpr int kScanWaves = 16;
constexpr int kScanSlice = kMaxGroups / kScanWaves;

__global__ __launch_bounds__(64 * kScanWaves) void k_group_scan(uint32_t* __restrict__ hist, int T,
                                                                int G, uint32_t* __restrict__ tot)
{
    __shared__ uint32_t s_sum[kScanWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int gq = (G + kScanWaves - 1) / kScanWaves, g0 = w * gq;
    uint32_t x[kScanSlice];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanSlice; ++j) {
        const int g = g0 + j;
        x[j] = (j < gq && g < G && t < T) ? hist[(int64_t)g * T + t] : 0u;
        sum += x[j];
    }
    s_sum[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, all = 0;
#pragma unroll
    for (int j = 0; j < kScanWaves; ++j) {
        const uint32_t y = s_sum[j][lane];
        run += j < w ? y : 0u;
        all += y;
    }
#pragma unroll
    for (int j = 0; j < kScanSlice; ++j) {
        const int g = g0 + j;
        if (j < gq && g < G && t < T) {
            hist[(int64_t)g * T + t] = run;
            run += x[j];
        }
    }
    if (w == 0 && t < T) tot[t] = all;
}

// One workgroup: the totals (M, min(M, capacity), overflow, N_v), the ranges
// of the T tiles from the exclusive scan of their totals (clamped to the
// capacity; an empty tile's range is (0, 0)), and the longest-first order of
// the first n tiles.  tot[t] is replaced by the tile's unclamped start.
constexpr int kRangeSlice = kGroupTiles / kOrderThreads;   // tiles per thread
static_assert(kRangeSlice * kOrderThreads == kGroupTiles, "whole slices");
static_assert(kMaxGroups <= kOrderThreads, "one group total per thread");

__global__ __launch_bounds__(kOrderThreads) void k_group_ranges(
    uint32_t* __restrict__ tot, int T, const uint32_t* __restrict__ d_tiles,
    const uint32_t* __restrict__ grp, int G, uint64_t capacity, uint32_t* __restrict__ ranges,
    uint32_t* __restrict__ order, uint32_t* __restrict__ n_long, uint32_t* __restrict__ n_huge,
    uint32_t* __restrict__ d_M, uint32_t* __restrict__ d_sortn, uint32_t* __restrict__ d_ovf,
    uint32_t* __restrict__ d_Nv)
{
    extern __shared__ uint32_t s_len[];   // [T] clamped list lengths
    __shared__ OrderSmem sm;
    __shared__ uint32_t s_tmp[kOrderThreads / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int t0 = tid * kRangeSlice;   // this thread's slice of tiles
    uint32_t c[kRangeSlice];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kRangeSlice; ++r) {
        c[r] = t0 + r < T ? tot[t0 + r] : 0u;
        s += c[r];
    }
    uint32_t nv = tid < G ? grp[G + tid] : 0u;
    uint32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
        nv += __shfl_xor(nv, d, 64);
    }
    if (lane == 63) {
        s_tmp[w][0] = inc;
        s_tmp[w][1] = nv;
    }
    __syncthreads();
    uint64_t start = inc - s, M = 0;
    uint32_t NV = 0;
    for (int j = 0; j < kOrderThreads / 64; ++j) {
        start += j < w ? s_tmp[j][0] : 0u;
        M += s_tmp[j][0];
        NV += s_tmp[j][1];
    }
#pragma unroll
    for (int r = 0; r < kRangeSlice; ++r) {
        const int t = t0 + r;
        if (t < T) {
            const uint64_t end = start + c[r];
            tot[t] = (uint32_t)start;
            uint32_t a = (uint32_t)min(start, capacity), b = (uint32_t)min(end, capacity);
            if (a == b) a = b = 0u;
            ranges[2 * t] = a;
            ranges[2 * t + 1] = b;
            s_len[t] = b - a;
            start = end;
        }
    }
    if (tid == 0) {
        *d_M = (uint32_t)M;
        *d_sortn = (uint32_t)min(M, capacity);
        *d_ovf = M > capacity ? 1u : 0u;
        *d_Nv = NV;
    }
    __syncthreads();
    const int n = d_tiles ? (int)min(*d_tiles, (uint32_t)T) : T;
    order_tiles(n, [&](int t) { return s_len[t]; }, order, n_long, n_huge, sm);
}

// Per group: every instance goes to its tile's start + the group's offset in
// the tile + the group's running count of the tile (LDS cursor); instances at
// or past the capacity are dropped, as the clamped ranges say.
__global__ __launch_bounds__(kGroupThreads) void k_group_place(
    const uint32_t* __restrict__ ntiles, const uint2* __restrict__ rect, int64_t N_host,
    const uint32_t* __restrict__ d_n, int tiles_x, const ts_view* __restrict__ views,
    int64_t per_view, int T, int G, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ start, uint64_t capacity, uint32_t* __restrict__ vals)
{
    extern __shared__ uint32_t s_cur[];   // [T]
    const int tid = threadIdx.x, g = xcd_group(G);
    const uint32_t cap = capacity < 0xffffffffull ? (uint32_t)capacity : 0xffffffffu;
    const int64_t N = d_n ? (int64_t)*d_n : N_host;
    int64_t e0, e1;
    group_span(N, G, g, e0, e1);
    const uint32_t* row = hist + (int64_t)g * T;
    for (int t = tid; t < T; t += kGroupThreads) s_cur[t] = start[t] + row[t];
    __syncthreads();
    for (int64_t e = e0 + (int64_t)tid * kGroupRun; e < e1;
         e += (int64_t)kGroupThreads * kGroupRun) {
        uint32_t n[kGroupRun];
        uint2 rb[kGroupRun];
        load_run(ntiles, rect, e, e1, n, rb);
        for_run_tiles(e, n, rb, tiles_x, views, per_view, [&](uint32_t t, uint32_t id) {
            if (t < (uint32_t)T) {
                const uint32_t p = atomicAdd(&s_cur[t], 1u);
                if (p < cap) vals[p] = id;
            }
        });
    }
}

// ---------------------------------------------------------------------------
// 4. per-tile depth order
// ---------------------------------------------------------------------------
struct SortSmem {   // the huge-tile block sort's digit counters
    uint16_t cnt[kItems * 4][kRadix];
    uint32_t base[kRadix];
    uint32_t tmp[4];
    uint32_t band, bor;
};

__device__ __forceinline__ uint64_t tile_key(uint32_t t, uint32_t depth_bits)
{
    return ((uint64_t)t << 32) | (uint64_t)depth_bits;
}

// Stable ranks inside one chunk of up to kChunk keys held striped: key[r] is
// item r * 256 + tid, present when that is below n.  Afterwards
// s.cnt[r * 4 + w][d] is the number of keys of digit d in the (round, wave)
// groups before (r, w), rank[r] the position of item r among the keys of its
// digit in its own group, and the result the chunk's count of digit `tid`.
template <class Smem>   // any shared struct with cnt[kItems * 4][kRadix]
__device__ uint32_t rank_chunk(const uint32_t (&key)[kItems], int n, int shift, Smem& s,
                               uint32_t (&rank)[kItems])
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slots = ((n + kBlock - 1) / kBlock) * 4;
    for (int q = 0; q < slots; ++q) s.cnt[q][tid] = 0;
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (r * kBlock < n) {   // the same for the whole block
            const bool ok = r * kBlock + tid < n;
            const uint32_t d = (key[r] >> shift) & 0xffu;
            uint64_t m = __ballot(ok);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool set = (d >> bit) & 1u;
                const uint64_t bal = __ballot(set);
                m &= set ? bal : ~bal;
            }
            rank[r] = (uint32_t)__popcll(m & lt);
            if (ok && (m & lt) == 0ull) s.cnt[r * 4 + w][d] = (uint16_t)__popcll(m);
        }
    }
    __syncthreads();
    uint32_t run = 0;
    for (int q = 0; q < slots; ++q) {
        const uint32_t c = s.cnt[q][tid];
        s.cnt[q][tid] = (uint16_t)run;
        run += c;
    }
    __syncthreads();
    return run;
}

// The bits in which the keys of the tile differ (block-wide AND / OR).
__device__ uint32_t varying_bits(uint32_t a, uint32_t o, SortSmem& s)
{
    if (threadIdx.x == 0) {
        s.band = ~0u;
        s.bor = 0u;
    }
    __syncthreads();
    atomicAnd(&s.band, a);
    atomicOr(&s.bor, o);
    __syncthreads();
    const uint32_t diff = s.band ^ s.bor;
    __syncthreads();
    return diff;
}

// L > 4 kWaveMax: each pass histograms the whole tile, then scatters it chunk by
// chunk in order between two global buffers (k1/v1, k0/v0 at the tile's own
// offsets); the last pass writes vals.  A single pass goes through k1/v1 and
// is copied back, so no pass reads and writes the same buffer.  A list that
// is not in index order (by_index) is first sorted by the triangle index, in
// passes over its varying bytes, so the depth passes see it in index order.
__device__ void sort_tile_large(int64_t L, uint32_t s0, uint32_t t, const float* depth,
                                uint32_t* vals, uint64_t* keys, uint32_t* k0, uint32_t* v0,
                                uint32_t* k1, uint32_t* v1, SortSmem& sm, bool by_index)
{
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t a = ~0u, o = 0u, ai = ~0u, oi = 0u;
    for (int64_t j = tid; j < L; j += kBlock) {
        const uint32_t v = vals[s0 + j];
        const uint32_t k = __float_as_uint(depth[v]);
        a &= k;
        o |= k;
        ai &= v;
        oi |= v;
    }
    const uint32_t diff = varying_bits(a, o, sm);
    const uint32_t diff_i = by_index ? varying_bits(ai, oi, sm) : 0u;
    uint32_t pmask = 0;   // digits that need a pass: bits 0-3 index bytes, 4-7 depth bytes
    for (int p = 0; p < 4; ++p) {
        if (((diff_i >> (8 * p)) & 0xffu) != 0u) pmask |= 1u << p;
        if (((diff >> (8 * p)) & 0xffu) != 0u) pmask |= 1u << (p + 4);
    }
    const int np = __popc(pmask);
    if (np == 0) {
        if (keys)
            for (int64_t j = tid; j < L; j += kBlock)
                keys[s0 + j] = tile_key(t, __float_as_uint(depth[vals[s0 + j]]));
        return;
    }
    const uint32_t* sk = nullptr;   // null: keys gathered from depth (or the index itself)
    const uint32_t* sv = vals + s0;
    for (int p = 0, q = 0; p < 8; ++p) {
        if (((pmask >> p) & 1u) == 0u) continue;
        const bool idx = p < 4;   // a pass over an index byte: the key is the value
        const int shift = 8 * (p & 3);
        const bool last = q == np - 1 && np > 1;
        uint32_t* dk = last ? nullptr : ((q & 1) ? k0 : k1) + s0;
        uint32_t* dv = last ? vals + s0 : ((q & 1) ? v0 : v1) + s0;
        sm.base[tid] = 0u;
        __syncthreads();
        for (int64_t j = tid; j < L; j += kBlock) {
            const uint32_t k = idx ? sv[j] : sk ? sk[j] : __float_as_uint(depth[sv[j]]);
            atomicAdd(&sm.base[(k >> shift) & 0xffu], 1u);
        }
        __syncthreads();
        const uint32_t h = sm.base[tid];
        uint32_t tot;
        const uint32_t pre = block_exclusive_scan(h, tot, sm.tmp);
        sm.base[tid] = pre;
        __syncthreads();
        for (int64_t c0 = 0; c0 < L; c0 += kChunk) {
            const int n = (int)min<int64_t>(kChunk, L - c0);
            uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
            for (int r = 0; r < kItems; ++r) {
                const int j = r * kBlock + tid;
                key[r] = 0u;
                val[r] = 0u;
                rank[r] = 0u;
                if (j < n) {
                    val[r] = sv[c0 + j];
                    key[r] = idx ? val[r] : sk ? sk[c0 + j] : __float_as_uint(depth[val[r]]);
                }
            }
            const uint32_t cnt = rank_chunk(key, n, shift, sm, rank);
#pragma unroll
            for (int r = 0; r < kItems; ++r) {
                const int j = r * kBlock + tid;
                if (j < n) {
                    const uint32_t d = (key[r] >> shift) & 0xffu;
                    const uint32_t pos = sm.base[d] + sm.cnt[r * 4 + w][d] + rank[r];
                    if (dk && !idx) dk[pos] = key[r];
                    dv[pos] = val[r];
                    if (last && keys)
                        keys[s0 + pos] =
                            tile_key(t, idx ? __float_as_uint(depth[val[r]]) : key[r]);
                }
            }
            __syncthreads();
            sm.base[tid] += cnt;
            __syncthreads();
        }
        sk = idx ? nullptr : dk;
        sv = dv;
        ++q;
    }
    if (np == 1)
        for (int64_t j = tid; j < L; j += kBlock) {
            const uint32_t v = v1[s0 + j];
            vals[s0 + j] = v;
            if (keys) keys[s0 + j] = tile_key(t, __float_as_uint(depth[v]));
        }
}

// ---- one wave per tile (L <= kWaveSortMax), or per quarter of a longer one --

// 32 KB: five workgroups fit in a CU's 160 KB of LDS
union TileSortSmem {
    SortSmem blk;
    uint64_t kv[(kBlock / 64) * kWaveMax];   // a long tile's four sorted quarters, merged in place
};
static_assert(sizeof(TileSortSmem) <= 32768, "five workgroups per CU");


// Bitonic sort of one tile's L <= 64 K entries by one wave, K entries per
// lane in registers: entry e = lane * K + r is the 64-bit key (depth bits <<
// 32 | triangle index), unique, so the network's (unstable) result is the
// (depth, index) order; slots past L hold the largest key.  Compare-exchange
// partners e ^ mask with mask < K are in the lane's own registers, the others
// come from lane ^ (mask / K) through a DPP move, a swizzle or a permute.  No
// LDS and no barriers, and fewer instructions than four 8-bit counting
// passes with their per-digit ballots (binning 0.1287 -> 0.1259 ms on the
// 3M-triangle view).
// The value of lane ^ D: DPP moves inside a 16-lane row (1: quad swap of
// pairs, 2: of halves, 3: quad reverse, 4: half-row mirror then quad reverse,
// 7: half-row mirror, 8: row rotate by 8, 15: row mirror), a swizzle inside
// a half-wave (16, 31), a permute through the LDS crossbar across halves
// (32, 63).
template <int D>
__device__ __forceinline__ int lane_xor32(int v)
{
    if constexpr (D == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, true);
    else if constexpr (D == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, true);
    else if constexpr (D == 3) return __builtin_amdgcn_mov_dpp(v, 0x1B, 0xf, 0xf, true);
    else if constexpr (D == 4)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, true), 0x1B,
                                        0xf, 0xf, true);
    else if constexpr (D == 7) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, true);
    else if constexpr (D == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, true);
    else if constexpr (D == 15) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, true);
    else if constexpr (D == 16 || D == 31) return __builtin_amdgcn_ds_swizzle(v, (D << 10) | 0x1F);
    else return __shfl_xor(v, D, 64);
}

template <int D>
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x)
{
    const int lo = lane_xor32<D>((int)(uint32_t)x);
    const int hi = lane_xor32<D>((int)(uint32_t)(x >> 32));
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One step of the network, then the rest of it, unrolled at compile time.
// The ascending form without directions: the first step of the merge of
// blocks of SIZE pairs e with e ^ (SIZE - 1), the later ones e with
// e ^ STRIDE; the smaller element always goes to the lower position.
template <int K, int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_stages(uint64_t (&x)[K], int lane)
{
    if constexpr (SIZE <= 64 * K) {
        constexpr bool flip = STRIDE == SIZE / 2;
        constexpr int MASK = flip ? SIZE - 1 : STRIDE;   // partner = e ^ MASK
        if constexpr (MASK < K) {   // both elements in this lane
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int q = r ^ MASK;
                if (r < q) {
                    const uint64_t a = x[r], b = x[q];
                    const bool lt = a < b;
                    x[r] = lt ? a : b;
                    x[q] = lt ? b : a;
                }
            }
        } else {                    // the partner is in lane ^ (MASK / K)
            constexpr int LD = MASK / K;              // 2^j - 1 (flip) or 2^j
            constexpr int HB = flip ? (LD + 1) / 2 : LD;   // the lane bit that orders the pair
            const bool lower = (lane & HB) == 0;
            uint64_t y[K];
#pragma unroll
            for (int r = 0; r < K; ++r) y[r] = shfl_xor64<LD>(x[flip ? K - 1 - r : r]);
#pragma unroll
            for (int r = 0; r < K; ++r) x[r] = (lower == (x[r] < y[r])) ? x[r] : y[r];
        }
        if constexpr (STRIDE > 1) bitonic_stages<K, SIZE, STRIDE / 2>(x, lane);
        else bitonic_stages<K, SIZE * 2, SIZE>(x, lane);
    }
}

// Loads the L <= 64 K entries vals[b ..] as keys (pads: the largest key) and
// sorts them with the wave's register network.
template <int K>
__device__ __forceinline__ void wave_sorted(int L, uint32_t b, const float* __restrict__ depth,
                                            const uint32_t* __restrict__ vals, uint64_t (&x)[K])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int e = lane * K + r;
        x[r] = ~0ull;
        if (e < L) {
            const uint32_t v = vals[b + e];
            x[r] = ((uint64_t)__float_as_uint(depth[v]) << 32) | v;
        }
    }
    bitonic_stages<K, 2, 1>(x, lane);
}

template <int K>
__device__ void bitonic_tile(int L, uint32_t s0, uint32_t t, const float* __restrict__ depth,
                             uint32_t* __restrict__ vals, uint64_t* __restrict__ keys)
{
    const int lane = threadIdx.x & 63;
    uint64_t x[K];
    wave_sorted<K>(L, s0, depth, vals, x);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int e = lane * K + r;
        if (e < L) {
            vals[s0 + e] = (uint32_t)x[r];
            if (keys) keys[s0 + e] = tile_key(t, (uint32_t)(x[r] >> 32));
        }
    }
}

// The wave-level sort: the smallest network that holds the tile.
__device__ void sort_tile_bitonic(int L, uint32_t s0, uint32_t t, const float* __restrict__ depth,
                                  uint32_t* __restrict__ vals, uint64_t* __restrict__ keys)
{
    if (L <= 64) bitonic_tile<1>(L, s0, t, depth, vals, keys);
    else if (L <= 128) bitonic_tile<2>(L, s0, t, depth, vals, keys);
    else if (L <= 256) bitonic_tile<4>(L, s0, t, depth, vals, keys);
    else if (L <= 512) bitonic_tile<8>(L, s0, t, depth, vals, keys);
    else bitonic_tile<16>(L, s0, t, depth, vals, keys);
}

// The non-flip steps of strides STRIDE, STRIDE / 2, ..., 1 on a wave's 64 K
// keys (layout as in bitonic_stages): the end of a merge whose first steps
// crossed waves.
template <int K, int STRIDE>
__device__ __forceinline__ void half_clean(uint64_t (&x)[K], int lane)
{
    if constexpr (STRIDE < K) {   // both elements in this lane
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int q = r ^ STRIDE;
            if (r < q) {
                const uint64_t a = x[r], b = x[q];
                const bool lt = a < b;
                x[r] = lt ? a : b;
                x[q] = lt ? b : a;
            }
        }
    } else {
        constexpr int LD = STRIDE / K;
        const bool lower = (lane & LD) == 0;
        uint64_t y[K];
#pragma unroll
        for (int r = 0; r < K; ++r) y[r] = shfl_xor64<LD>(x[r]);
#pragma unroll
        for (int r = 0; r < K; ++r) x[r] = (lower == (x[r] < y[r])) ? x[r] : y[r];
    }
    if constexpr (STRIDE > 1) half_clean<K, STRIDE / 2>(x, lane);
}

// LDS slot of key e of a long tile: inside each run of K keys (one lane's)
// the slot is XORed with the lane's low bits, so the lanes of a wave storing
// their r-th keys hit different banks.
template <int K>
__device__ __forceinline__ int kv_slot(int e)
{
    return e ^ ((e / K) & (K - 1));
}

// One merge step over the workgroup's N keys in LDS: the pairs (e, e ^ (S-1))
// of every block of S (flip) or (e, e + S) (stride S), smaller key first.
template <int K, bool FLIP>
__device__ __forceinline__ void lds_step(uint64_t* __restrict__ kv, int S, int N)
{
    const int half = FLIP ? S >> 1 : S;
    for (int p = threadIdx.x; p < N / 2; p += kBlock) {
        const int off = p & (half - 1), blk = p - off;
        const int i = 2 * blk + off;
        const int j = FLIP ? 2 * blk + S - 1 - off : i + S;
        const int si = kv_slot<K>(i), sj = kv_slot<K>(j);
        const uint64_t a = kv[si], b = kv[sj];
        if (b < a) {
            kv[si] = b;
            kv[sj] = a;
        }
    }
}

// A long tile: wave w sorts quarter w (entries w * Qa .. of the tile, Qa =
// ceil(L / 4)) with the register network, padded to Q = 64 K keys with the
// largest one; the last two levels of the same direction-free network merge
// the four runs.  Only their steps whose pairs cross waves (each level's
// first, and stride Q of the last) go through LDS; the rest run in registers.
template <int K>
__device__ void sort_long_tile(int L, uint32_t s0, uint32_t t, const float* __restrict__ depth,
                               uint32_t* __restrict__ vals, uint64_t* __restrict__ keys,
                               uint64_t* __restrict__ kv)
{
    constexpr int Q = 64 * K, N = 4 * Q;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int Qa = (L + 3) >> 2;
    const int q0 = w * Qa;
    uint64_t x[K];
    wave_sorted<K>(max(0, min(Qa, L - q0)), s0 + (uint32_t)q0, depth, vals, x);
    uint64_t* mine = kv + w * Q + lane * K;   // key r of this lane at mine[r ^ sw]
    const int sw = lane & (K - 1);
    // level 2Q: the flip pairs waves 0-1 and 2-3, then strides Q/2 .. 1
#pragma unroll
    for (int r = 0; r < K; ++r) mine[r ^ sw] = x[r];
    __syncthreads();
    lds_step<K, true>(kv, 2 * Q, N);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < K; ++r) x[r] = mine[r ^ sw];
    half_clean<K, Q / 2>(x, lane);
    // level 4Q: the flip and stride Q cross waves, then strides Q/2 .. 1
#pragma unroll
    for (int r = 0; r < K; ++r) mine[r ^ sw] = x[r];
    __syncthreads();
    lds_step<K, true>(kv, 4 * Q, N);
    __syncthreads();
    lds_step<K, false>(kv, Q, N);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < K; ++r) x[r] = mine[r ^ sw];
    half_clean<K, Q / 2>(x, lane);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int e = w * Q + lane * K + r;
        if (e < L) {
            vals[s0 + e] = (uint32_t)x[r];
            if (keys) keys[s0 + e] = tile_key(t, (uint32_t)(x[r] >> 32));
        }
    }
}

// Tiles taken in `order` (longest first); the first n_long of them are longer
// than kWaveSortMax and get a whole workgroup each (four wave-level sorts of a
// quarter each and a two-level merge up to 4 kWaveMax entries, global
// ping-pong or the segmented sort beyond); every later workgroup gives each of its four
// waves one tile.  The instances of a tile arrive in index order, or in any
// order when `unordered` is set; they leave in (depth, index) order, with
// their 64-bit keys when keys is set.
__global__ __launch_bounds__(256) void k_tile_sort(const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ n_long,
                                                   int num_tiles,
                                                   const uint32_t* __restrict__ d_tiles,
                                                   const float* __restrict__ depth,
                                                   uint32_t* __restrict__ vals,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ k0,
                                                   uint32_t* __restrict__ v0,
                                                   uint32_t* __restrict__ k1,
                                                   uint32_t* __restrict__ v1, int segmented,
                                                   int unordered)
{
    __shared__ TileSortSmem sm;
    const uint32_t n = d_tiles ? min(*d_tiles, (uint32_t)num_tiles) : (uint32_t)num_tiles;
    const uint32_t nl = min(*n_long, n);
    uint32_t idx;
    if (blockIdx.x < nl) {
        idx = blockIdx.x;
    } else {
        idx = nl + (blockIdx.x - nl) * (kBlock / 64) + (threadIdx.x >> 6);
        if (idx >= n) return;   // whole waves leave; no workgroup barrier follows
    }
    const uint32_t t = order[idx];
    if (t >= (uint32_t)num_tiles) return;
    const uint32_t s0 = ranges[2 * t];
    const int64_t L = (int64_t)ranges[2 * t + 1] - (int64_t)s0;
    if (blockIdx.x < nl && L > kHugeLen) {   // the whole workgroup, in global memory
        if (!segmented)
            sort_tile_large(L, s0, t, depth, vals, keys, k0, v0, k1, v1, sm.blk, unordered != 0);
        return;   // else the segmented sort below takes the tile
    }
    if (blockIdx.x < nl) {   // the whole workgroup: four quarters and a merge
        if (L <= 4 * 64) sort_long_tile<1>((int)L, s0, t, depth, vals, keys, sm.kv);
        else if (L <= 4 * 128) sort_long_tile<2>((int)L, s0, t, depth, vals, keys, sm.kv);
        else if (L <= 4 * 256) sort_long_tile<4>((int)L, s0, t, depth, vals, keys, sm.kv);
        else if (L <= 4 * 512) sort_long_tile<8>((int)L, s0, t, depth, vals, keys, sm.kv);
        else sort_long_tile<16>((int)L, s0, t, depth, vals, keys, sm.kv);
        return;
    }
    // one wave-level sort per wave: a whole tile
    if (L == 1) {
        if (keys && (threadIdx.x & 63) == 0)
            keys[s0] = tile_key(t, __float_as_uint(depth[vals[s0]]));
    } else if (L > 1 && L <= kWaveSortMax) {
        sort_tile_bitonic((int)L, s0, t, depth, vals, keys);
    }
}

// ---------------------------------------------------------------------------
// 4b. segmented depth sort of the tiles longer than kHugeLen entries: every
// pass spreads each such tile over many workgroups (one per kChunk entries),
// as the global passes of step 3 do -- per-chunk digit histograms, a scan per
// tile over (digit, chunk), a stable scatter -- instead of one workgroup per
// tile walking its chunks in turn.
// ---------------------------------------------------------------------------

// The huge tiles, listed from the first n_long entries of the order (they
// lead it), and the prefix of their chunk counts: hl[k], cst[k] for k < nh,
// cst[nh] = all chunks, cst[nh + 1] = nh.
__global__ __launch_bounds__(kOrderThreads) void k_seg_plan(const uint32_t* __restrict__ ranges,
                                                            const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ n_long,
                                                            int num_tiles,
                                                            uint32_t* __restrict__ hl,
                                                            uint32_t* __restrict__ cst)
{
    __shared__ uint32_t s_w[kOrderThreads / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nl = min(*n_long, (uint32_t)num_tiles);
    uint32_t run_n = 0, run_c = 0;   // the same in every thread
    for (uint32_t base = 0; base < nl; base += kOrderThreads) {
        const uint32_t i = base + tid;
        uint32_t t = 0, L = 0;
        if (i < nl) {
            t = order[i];
            if (t < (uint32_t)num_tiles) L = ranges[2 * t + 1] - ranges[2 * t];
        }
        const uint32_t huge = L > (uint32_t)kHugeLen ? 1u : 0u;
        const uint32_t ch = huge ? (L + kChunk - 1) / kChunk : 0u;
        uint32_t a = huge, b = ch;   // inclusive wave scans
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ya = __shfl_up(a, d, 64), yb = __shfl_up(b, d, 64);
            a += lane >= d ? ya : 0u;
            b += lane >= d ? yb : 0u;
        }
        if (lane == 63) {
            s_w[w][0] = a;
            s_w[w][1] = b;
        }
        __syncthreads();
        uint32_t pa = 0, pb = 0, ta = 0, tb = 0;
        for (int k = 0; k < kOrderThreads / 64; ++k) {
            pa += k < w ? s_w[k][0] : 0u;
            pb += k < w ? s_w[k][1] : 0u;
            ta += s_w[k][0];
            tb += s_w[k][1];
        }
        if (huge) {
            const uint32_t k = run_n + pa + a - 1;
            hl[k] = t;
            cst[k] = run_c + pb + b - ch;
        }
        run_n += ta;
        run_c += tb;
        __syncthreads();
    }
    if (tid == 0) {
        cst[run_n] = run_c;
        cst[num_tiles + 1] = run_n;
    }
}

// The chunk c of the segmented list: its huge tile k and its element range.
struct SegChunk {
    uint32_t t, s0, lo, n;
    int k;
};

__device__ __forceinline__ bool seg_chunk(uint32_t c, const uint32_t* __restrict__ hl,
                                          const uint32_t* __restrict__ cst, int num_tiles,
                                          const uint32_t* __restrict__ ranges, SegChunk& q)
{
    const uint32_t nh = cst[num_tiles + 1];
    if (nh == 0u || c >= cst[nh]) return false;
    int lo = 0, hi = (int)nh - 1;   // the last k with cst[k] <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cst[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    q.k = lo;
    q.t = hl[lo];
    q.s0 = ranges[2 * q.t];
    const uint32_t L = ranges[2 * q.t + 1] - q.s0;
    q.lo = (c - cst[lo]) * (uint32_t)kChunk;
    q.n = min((uint32_t)kChunk, L - q.lo);
    return true;
}

// Per-chunk digit histogram.  The first pass (kin null) gathers the keys from
// depth and, when kfirst is set, keeps them there at the entries' positions,
// so its scatter reads them in order instead of gathering them again; later
// passes read only the keys.
__global__ __launch_bounds__(kBlock) void k_seg_hist(const uint32_t* __restrict__ hl,
                                                     const uint32_t* __restrict__ cst,
                                                     int num_tiles,
                                                     const uint32_t* __restrict__ ranges,
                                                     const uint32_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     const float* __restrict__ depth, int shift,
                                                     uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ kfirst)
{
    __shared__ uint32_t h[kRadix];
    SegChunk q;
    if (!seg_chunk(blockIdx.x, hl, cst, num_tiles, ranges, q)) return;
    h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t j = (uint32_t)(r * kBlock + threadIdx.x);
        if (j < q.n) {
            const uint32_t pos = q.s0 + q.lo + j;
            uint32_t key;
            if (kin) {
                key = kin[pos];
            } else {
                key = __float_as_uint(depth[vin[pos]]);
                if (kfirst) kfirst[pos] = key;
            }
            atomicAdd(&h[(key >> shift) & 0xffu], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)blockIdx.x * kRadix + threadIdx.x] = h[threadIdx.x];   // chunk-major
}

// One workgroup per huge tile, one thread per digit: the offsets of every
// (digit, chunk) of the tile, in digit-major, chunk-minor order, written over
// the histogram (chunk-major rows of 256 digits: each step of a thread's walk
// over the chunks is one coalesced row access of the workgroup).
__global__ __launch_bounds__(kBlock) void k_seg_scan(const uint32_t* __restrict__ hl,
                                                     const uint32_t* __restrict__ cst,
                                                     int num_tiles,
                                                     const uint32_t* __restrict__ ranges,
                                                     uint32_t* __restrict__ hist)
{
    __shared__ uint32_t tmp[4];
    const uint32_t nh = cst[num_tiles + 1];
    const uint32_t k = blockIdx.x;
    if (k >= nh) return;
    const uint32_t c0 = cst[k], c1 = cst[k + 1];
    const uint32_t s0 = ranges[2 * hl[k]];
    uint32_t* hd = hist + threadIdx.x;
    uint32_t tot = 0;
#pragma unroll 8
    for (uint32_t c = c0; c < c1; ++c) tot += hd[(int64_t)c * kRadix];
    uint32_t all;
    uint32_t base = s0 + block_exclusive_scan(tot, all, tmp);
#pragma unroll 8
    for (uint32_t c = c0; c < c1; ++c) {
        const uint32_t x = hd[(int64_t)c * kRadix];
        hd[(int64_t)c * kRadix] = base;
        base += x;
    }
}

// Stable scatter of one chunk of a huge tile, ranked and written as in
// k_radix_scatter: wave w ranks the chunk's entries w * 512 + r * 64 + lane
// (the leader of a group takes the count of its digit in the wave's earlier
// rounds from the return value of its LDS add), the chunk is placed in LDS in
// sorted order and written out by consecutive lanes.  Positions start at the
// chunk's offsets from the scanned (digit, chunk) histogram of its tile.
__global__ __launch_bounds__(kBlock) void k_seg_scatter(
    const uint32_t* __restrict__ hl, const uint32_t* __restrict__ cst, int num_tiles,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ kin,
    const uint32_t* __restrict__ vin, const float* __restrict__ depth, int shift,
    const uint32_t* __restrict__ hist, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, uint64_t* __restrict__ keys)
{
    constexpr int kWaveKeys = kChunk / (kBlock / 64);   // 512 entries per wave
    __shared__ uint32_t s_off[kRadix];   // output position of the chunk's k-th entry of digit d: s_off[d] + k
    __shared__ uint32_t s_lst[kRadix];   // first LDS slot of digit d
    __shared__ uint32_t s_cnt[kBlock / 64][kRadix];   // per wave and digit: count, then the waves before
    __shared__ uint32_t s_key[kChunk];
    __shared__ uint32_t s_val[kChunk];
    __shared__ uint32_t s_tmp[4];
    SegChunk q;
    if (!seg_chunk(blockIdx.x, hl, cst, num_tiles, ranges, q)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nloc = (int)q.n;
#pragma unroll
    for (int c = 0; c < kBlock / 64; ++c) s_cnt[c][tid] = 0u;
    __syncthreads();

    uint32_t key[kItems], val[kItems], within[kItems];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int j = w * kWaveKeys + r * 64 + lane;
        const bool ok = j < nloc;
        key[r] = 0u;
        val[r] = 0u;
        if (ok) {
            const uint32_t pos = q.s0 + q.lo + (uint32_t)j;
            val[r] = vin[pos];
            key[r] = kin ? kin[pos] : __float_as_uint(depth[val[r]]);
        }
        const uint32_t d = (key[r] >> shift) & 0xffu;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t bal = __ballot(set);
            m &= set ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t lead = m != 0ull ? (uint32_t)__builtin_ctzll(m) : (uint32_t)lane;
        uint32_t before = 0u;
        if (ok && rank == 0u) before = atomicAdd(&s_cnt[w][d], (uint32_t)__popcll(m));
        within[r] = (uint32_t)__shfl((int)before, (int)lead, 64) + rank;
    }
    __syncthreads();
    uint32_t run = 0;
#pragma unroll
    for (int c = 0; c < kBlock / 64; ++c) {
        const uint32_t x = s_cnt[c][tid];
        s_cnt[c][tid] = run;
        run += x;
    }
    uint32_t btot;
    const uint32_t lstart = block_exclusive_scan(run, btot, s_tmp);   // barriers inside
    s_lst[tid] = lstart;
    // the chunk's first position for each digit, from the scanned histogram
    s_off[tid] = hist[(int64_t)blockIdx.x * kRadix + tid] - lstart;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (w * kWaveKeys + r * 64 + lane < nloc) {
            const uint32_t d = (key[r] >> shift) & 0xffu;
            const uint32_t slot = s_lst[d] + s_cnt[w][d] + within[r];
            s_key[slot] = key[r];
            s_val[slot] = val[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int j = r * kBlock + tid;
        if (j < nloc) {
            const uint32_t k = s_key[j];
            const uint32_t pos = s_off[(k >> shift) & 0xffu] + (uint32_t)j;
            if (kout) kout[pos] = k;
            vout[pos] = s_val[j];
            if (keys) keys[pos] = tile_key(q.t, k);
        }
    }
}

// ---------------------------------------------------------------------------

static hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                             uint32_t* kfin, uint32_t* vfin, const uint32_t* d_n,
                             int64_t n_max, int bits, const BinWorkspace& ws,
                             hipStream_t stream)
{
    const int passes = (bits + 7) / 8;
    const int dbits = (bits + passes - 1) / passes;   // <= 8: the bits split evenly
    const int64_t nb = nblocks(n_max > 0 ? n_max : 1);
    uint32_t* ks[2] = {k0, k1};
    uint32_t* vs[2] = {v0, v1};
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = dbits * p;
        const bool last = p == passes - 1;
        uint32_t* ko = last ? kfin : ks[src ^ 1];
        uint32_t* vo = last ? vfin : vs[src ^ 1];
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, stream, ks[src], d_n,
                           shift, dbits, ws.hist, ws.hist_stride);
        hipLaunchKernelGGL(k_radix_scan, dim3(1u << dbits), dim3(kBlock), 0, stream, ws.hist, d_n,
                           ws.hist_stride, ws.dtot);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, stream, ks[src],
                           vs[src], ko, vo, d_n, shift, dbits, ws.hist, ws.hist_stride, ws.dtot);
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
    const bool seg = (out.flags & TS_BINS_SEGMENTED_SORT) != 0u;
    uint32_t* order = out.order ? out.order : ws.torder;
    uint32_t* n_long = ws.ctl + 1;

    if (!seg && num_tiles > 0 && num_tiles <= kGroupTiles) {
        // 1'. group tile counts, column scan, ranges and order, placement
        const int64_t want = (N + kGroupEntries - 1) / kGroupEntries;
        const int G = want < 1 ? 1 : want > kMaxGroups ? kMaxGroups : (int)want;
        const size_t lds = 4 * (size_t)num_tiles;
        const uint2* r4 = reinterpret_cast<const uint2*>(rect);
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)G), dim3(kGroupThreads), lds, stream,
                           ntiles, r4, N, d_n, tiles_x, views, per_view, num_tiles, G, ws.hist,
                           ws.blk);
        hipLaunchKernelGGL(k_group_scan, dim3((unsigned)((num_tiles + 63) / 64)),
                           dim3(64 * kScanWaves), 0,
                           stream, ws.hist, num_tiles, G, ws.hl);
        hipLaunchKernelGGL(k_group_ranges, dim3(1), dim3(kOrderThreads), lds, stream,
                           ws.hl, num_tiles, d_tiles, (const uint32_t*)ws.blk, G,
                           out.capacity, out.ranges, order, n_long, out.d_count + 3, d_M, d_sortn,
                           d_ovf, d_Nv);
        hipLaunchKernelGGL(k_group_place, dim3((unsigned)G), dim3(kGroupThreads), lds, stream,
                           ntiles, r4, N, d_n, tiles_x, views, per_view, num_tiles, G,
                           (const uint32_t*)ws.hist, (const uint32_t*)ws.hl, out.capacity,
                           out.vals);
        // 4. depth order inside every tile
        hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)num_tiles), dim3(kBlock), 0, stream,
                           out.ranges, (const uint32_t*)order, (const uint32_t*)n_long, num_tiles,
                           d_tiles, depth, out.vals, out.keys, ws.tk[0], ws.tv[0], ws.tk[1],
                           ws.tv[1], 0, 1);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess || !h_count) return err;
        err = hipMemcpyAsync(h_count, out.d_count, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                             stream);
        if (err != hipSuccess) return err;
        err = hipStreamSynchronize(stream);
        if (err != hipSuccess) return err;
        *overflow = (uint64_t)h_count[0] > out.capacity;
        return hipSuccess;
    }

    // 1. tile counts of the N (or *d_n) entries in index order; ranges cleared
    hipLaunchKernelGGL(k_count, dim3((unsigned)nbN), dim3(kBlock), 0, stream, ntiles, N, d_n,
                       ws.blk, ws.blk_vis, out.ranges, 2 * (int64_t)num_tiles);
    // 2. instances in index order (up to capacity), and the totals
    hipLaunchKernelGGL(k_emit, dim3((unsigned)(nbN > 0 ? nbN : 1)), dim3(kBlock), 0, stream,
                       ntiles, reinterpret_cast<const short4*>(rect), N, d_n,
                       (const uint32_t*)ws.blk, (const uint32_t*)ws.blk_vis, tiles_x, views,
                       per_view, out.capacity, ws.tk[0], ws.tv[0], d_M, d_sortn, d_ovf, d_Nv);
    int64_t m_max = (int64_t)out.capacity;
    if (h_count) {
        hipError_t err = hipMemcpyAsync(h_count, out.d_count, 2 * sizeof(uint32_t),
                                        hipMemcpyDeviceToHost, stream);
        if (err != hipSuccess) return err;
        err = hipStreamSynchronize(stream);
        if (err != hipSuccess) return err;
        if ((uint64_t)h_count[0] > out.capacity) {
            // ranges are all empty here; keep the order valid for any raster
            // launched before the caller grows the list
            *overflow = true;
            launch_tile_order(out.ranges, num_tiles, d_tiles, out.order, stream, nullptr,
                              out.d_count + 3);
            return hipGetLastError();
        }
        m_max = h_count[0];
    }
    // 3. stable sort by tile, ranges, longest-first tile order
    hipError_t err = radix_sort(ws.tk[0], ws.tv[0], ws.tk[1], ws.tv[1], ws.tfin, out.vals,
                                d_sortn, m_max, bits_for(num_tiles), ws, stream);
    if (err != hipSuccess) return err;
    if (m_max > 0)
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((m_max + 255) / 256)), dim3(256), 0, stream,
                           ws.tfin, d_sortn, out.ranges);
    launch_tile_order(out.ranges, num_tiles, d_tiles, order, stream, n_long, out.d_count + 3);
    // 4. depth order inside every tile
    if (m_max > 0 && num_tiles > 0)
        hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)num_tiles), dim3(kBlock), 0, stream,
                           out.ranges, (const uint32_t*)order, (const uint32_t*)n_long, num_tiles,
                           d_tiles, depth, out.vals, out.keys, ws.tk[0], ws.tv[0], ws.tk[1],
                           ws.tv[1], seg ? 1 : 0, 0);
    if (seg && m_max > 0 && num_tiles > 0) {
        // 4b. the huge tiles, spread over many workgroups: four stable passes
        hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(kOrderThreads), 0, stream, out.ranges,
                           (const uint32_t*)order, (const uint32_t*)n_long, num_tiles, ws.hl,
                           ws.cst);
        const unsigned nc = (unsigned)(nblocks(m_max) + num_tiles);
        const uint32_t* kin = nullptr;
        const uint32_t* vin = out.vals;
        for (int p = 0; p < 4; ++p) {
            const bool last = p == 3;
            uint32_t* kout = last ? nullptr : ws.tk[(p + 1) & 1];
            uint32_t* vout = last ? out.vals : ws.tv[(p + 1) & 1];
            // the first pass keeps the gathered keys in tk[0], free until the
            // second pass writes it
            hipLaunchKernelGGL(k_seg_hist, dim3(nc), dim3(kBlock), 0, stream,
                               (const uint32_t*)ws.hl, (const uint32_t*)ws.cst, num_tiles,
                               out.ranges, kin, vin, depth, 8 * p, ws.hist,
                               p == 0 ? ws.tk[0] : nullptr);
            if (p == 0) kin = ws.tk[0];
            hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)num_tiles), dim3(kBlock), 0, stream,
                               (const uint32_t*)ws.hl, (const uint32_t*)ws.cst, num_tiles,
                               out.ranges, ws.hist);
            hipLaunchKernelGGL(k_seg_scatter, dim3(nc), dim3(kBlock), 0, stream,
                               (const uint32_t*)ws.hl, (const uint32_t*)ws.cst, num_tiles,
                               out.ranges, kin, vin, depth, 8 * p, (const uint32_t*)ws.hist,
                               kout, vout, last ? out.keys : nullptr);
            kin = kout;
            vin = vout;
        }
    }
    return hipGetLastError();
}

}  // namespace ts
