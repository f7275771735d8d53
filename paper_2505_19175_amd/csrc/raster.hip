// raster.hip -- per-tile compositing on gfx950: forward (front to back) and
// backward (back to front, transmittance recovered from the final value).
//
// One 256-thread workgroup per 16x16 tile.  Wave w owns the 8x8 quadrant
// (w & 1, w >> 1) and each of its four 16-lane rows (a DPP row) owns a 4x4
// block of it: lane l shades pixel (l & 3, (l >> 2) & 3) of block
// g = l >> 4 = (g & 1, g >> 1).
//
// The tile's list is walked in batches of 256 entries staged through LDS:
// each thread copies one record as six 16-byte chunks and its depth into
// chunk-major arrays (consecutive lanes write consecutive slots: no bank
// conflicts) and marks the 4x4 blocks of the tile that can hold a pixel it
// composites.  Each wave then writes, for each of its four blocks, the byte
// indices of the batch entries marked for it (ballot + mbcnt compaction), so
// every row walks its own list -- one wave step advances four lists, and a
// row never evaluates a triangle that misses its block.  The lists live in
// LDS and are read one byte per lane per step: no scalar list bookkeeping.
//
// The window is evaluated as three FP64 affine functions per pixel (gfx950
// issues v_fma_f64 at the rate of unpacked v_fma_f32); the rest is FP32,
// written without branches so a wave issues one path per step.  Every
// kernel is instantiated per window function (TS_WINDOW_*).
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kBatch = kBlock;   // entries staged per batch
constexpr int kChunks = 6;       // 16-byte chunks of a record the raster reads (+ z)

// phi_lse(s) of each staged entry, for the LogSumExp window only: the other
// windows get an empty base, so their LDS footprint (32000 bytes, 25 blocks
// of the 1280-byte allocation unit: five workgroups per CU) is unchanged.
template <int WIN>
struct StageExtra {
    static constexpr bool kLse = false;
};
template <>
struct StageExtra<TS_WINDOW_LSE> {
    static constexpr bool kLse = true;
    float ps[kBatch];
};

// The forward that keeps pruning statistics gathers them per batch entry in
// words the plain forward does not need during its walk, so its LDS stays at
// 25 allocation units: the largest T*o (float bits; non-negative floats
// order as integers) in the triangle-index words, the composited pixels as
// 16-bit halves of the per-entry block-hit words (dead once every wave has
// built its lists).  One global max and one add per entry and tile flush
// them at the end of the batch.
template <int WIN, bool ST = false>
struct StageT : StageExtra<WIN> {
    float4 q[kChunks][kBatch];
    float z[kBatch];
    uint16_t hit[kBatch];        // bit 4 w + g: may composite in block g of quadrant w
    uint8_t list[16][kBatch];    // per block 4 w + g: its entries of the batch, in order
    uint32_t comp[kBatch / 2];   // forward: blocks where each entry composited, 16 bits each
    uint32_t tri[kBatch];        // triangle (entry) index of each staged entry
};

union RecView {
    float4 q[8];
    TriRecord r;
};

// Copy record `tri` into LDS slot threadIdx.x and return the mask of the
// tile's sixteen 4x4 blocks that may hold a composited pixel of it: the
// tight box touches the block, and for every edge k the largest u_k over the
// block's pixel centres (at one corner, u_k being affine) reaches ut, the
// lower bound of u over pixels that composite.  The box and the three edge
// tests are the separating axes of the tight region (a triangle) and the
// block's square of pixel centres.  The slack covers the rounding of this
// evaluation and of the per-pixel one, so no pixel that composites is lost.
//
// The staged copy holds C_k relative to the tile's corner pixel (tx0, ty0)
// instead of the record's anchor, so a lane evaluates u_k = A_k dx + B_k dy +
// C_k with its own fixed offset in the tile (no per-step conversion).  The
// forward (ZA) needs no anchor after that: it stages the depth in the
// anchor's four bytes, so a step reads C[2], z and o with one 16-byte load.
template <bool ZA, class Stage>
__device__ __forceinline__ void write_stage(Stage& S, RecView& u, int tx0, int ty0)
{
    const double ox = (double)(tx0 - u.r.ax), oy = (double)(ty0 - u.r.ay);
#pragma unroll
    for (int k = 0; k < 3; ++k) u.r.C[k] = fma(u.r.A[k], ox, fma(u.r.B[k], oy, u.r.C[k]));
    if constexpr (ZA) u.q[4].z = u.r.z;   // bytes 72-75: the anchor
#pragma unroll
    for (int c = 0; c < kChunks; ++c) S.q[c][threadIdx.x] = u.q[c];
    if constexpr (!ZA) S.z[threadIdx.x] = u.r.z;
    if constexpr (Stage::kLse) S.ps[threadIdx.x] = u.r.phis;
}

template <bool ZA = false, class Stage>
__device__ __forceinline__ void stage_copy(Stage& S, const TriRecord* __restrict__ rec,
                                           uint32_t tri, int tx0, int ty0)
{
    const float4* src = reinterpret_cast<const float4*>(rec + tri);
    RecView u;
    constexpr int nc = Stage::kLse ? 8 : 7;   // phis sits in chunk 7
#pragma unroll
    for (int c = 0; c < nc; ++c) u.q[c] = src[c];
    write_stage<ZA>(S, u, tx0, ty0);
}

template <bool ZA = false, class Stage>
__device__ __forceinline__ uint32_t stage_rec(Stage& S, const TriRecord* __restrict__ rec,
                                              uint32_t tri, int tx0, int ty0)
{
    const float4* src = reinterpret_cast<const float4*>(rec + tri);
    RecView u;
#pragma unroll
    for (int c = 0; c < 8; ++c) u.q[c] = src[c];
    write_stage<ZA>(S, u, tx0, ty0);
    uint32_t cx = 0, cy = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x0 = tx0 + 4 * i, y0 = ty0 + 4 * i;
        cx |= (u.r.px0 <= x0 + 3 && u.r.px1 >= x0) ? (1u << i) : 0u;
        cy |= (u.r.py0 <= y0 + 3 && u.r.py1 >= y0) ? (1u << i) : 0u;
    }
    uint32_t box = 0;   // bit 4 by + bx
#pragma unroll
    for (int by = 0; by < 4; ++by) box |= ((cy >> by) & 1u) ? (cx << (4 * by)) : 0u;

    const double ut = (double)u.r.ut;
    // tile-relative coefficients read back from this thread's own LDS slot,
    // one edge at a time, to keep the register peak of the staging step low
    const double* cf = reinterpret_cast<const double*>(&S.q[0][0]);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        auto coef = [&](int idx) {   // double idx of the record: chunk idx / 2, half idx % 2
            return cf[2 * (size_t)((idx >> 1) * kBatch + threadIdx.x) + (idx & 1)];
        };
        const double A = coef(k), B = coef(3 + k), C = coef(6 + k);
        const double cxk = A > 0.0 ? 3.0 : 0.0, cyk = B > 0.0 ? 3.0 : 0.0;
        const double base = fma(A, cxk, fma(B, cyk, C));   // largest u_k over block (0, 0)
        const double slack = 0x1p-46 * (fabs(C) + 16.0 * (fabs(A) + fabs(B)));
        const double lim = ut - slack;
        const double A4 = 4.0 * A, B4 = 4.0 * B;
#pragma unroll 1
        for (int by = 0; by < 4; ++by) {
            const double rb = fma(B4, (double)by, base);
#pragma unroll
            for (int bx = 0; bx < 4; ++bx) {
                const double val = fma(A4, (double)bx, rb);
                box &= val >= lim ? ~0u : ~(1u << (4 * by + bx));
            }
        }
    }
    uint32_t m = 0;
#pragma unroll
    for (int by = 0; by < 4; ++by)
#pragma unroll
        for (int bx = 0; bx < 4; ++bx) {
            const int w = (bx >> 1) + 2 * (by >> 1), g = (bx & 1) + 2 * (by & 1);
            m |= ((box >> (4 * by + bx)) & 1u) << (4 * w + g);
        }
    return m;
}

template <bool ZA = false, class Stage>
__device__ __forceinline__ TriRecord read_rec(const Stage& S, int j)
{
    RecView u;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) u.q[c] = S.q[c][j];
    u.r.z = ZA ? u.q[4].z : S.z[j];
    if constexpr (Stage::kLse) u.r.phis = S.ps[j];
    return u.r;
}

// Write the entry lists of the wave's four blocks for a batch of n entries:
// S.list[4 w + g] receives, in increasing order, the entries e < lim_g whose
// mark for block g is set.  Returns the four lengths (wave-uniform).
struct Lens {
    int n0, n1, n2, n3;
};

template <class Stage>
__device__ __forceinline__ Lens build_lists(Stage& S, int n, int w, int lane, int lim0,
                                            int lim1, int lim2, int lim3)
{
    Lens L{0, 0, 0, 0};
    uint8_t* l0 = S.list[4 * w];
    uint8_t* l1 = S.list[4 * w + 1];
    uint8_t* l2 = S.list[4 * w + 2];
    uint8_t* l3 = S.list[4 * w + 3];
#pragma unroll
    for (int c = 0; c < kBatch / 64; ++c) {
        const int e = c * 64 + lane;
        const uint32_t h = e < n ? ((uint32_t)S.hit[e] >> (4 * w)) & 0xfu : 0u;
        auto put = [&](bool bit, uint8_t* lst, int& len) {
            const uint64_t m = __ballot(bit);
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (bit) lst[len + (int)below] = (uint8_t)e;
            len += __popcll(m);
        };
        put((h & 1u) && e < lim0, l0, L.n0);
        put((h & 2u) && e < lim1, l1, L.n1);
        put((h & 4u) && e < lim2, l2, L.n2);
        put((h & 8u) && e < lim3, l3, L.n3);
    }
    // the lists are read by other lanes of this wave only: order the byte
    // writes before those reads without a workgroup barrier
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return L;
}

__device__ __forceinline__ int per_row(int g, int j0, int j1, int j2, int j3)
{
    return g == 0 ? j0 : g == 1 ? j1 : g == 2 ? j2 : j3;
}

// min_k u_k without the arg-min, for the forward: one v_min_f64 per edge
// instead of a compare and two selects.  The three u_k are the same FMAs as
// in edge_min, so the minimum is the same double.
__device__ __forceinline__ double edge_min_value(const double* A, const double* B,
                                                 const double* C, double dx, double dy)
{
    const double u0 = fma(A[0], dx, fma(B[0], dy, C[0]));
    const double u1 = fma(A[1], dx, fma(B[1], dy, C[1]));
    const double u2 = fma(A[2], dx, fma(B[2], dy, C[2]));
    return fmin(fmin(u0, u1), u2);
}

// Window and opacity of a staged record at the pixel (dx, dy) from the
// tile's corner.  Returns whether the pixel is in the window's support (the
// forms of Eq. 1: u > 0; the sigmoid: everywhere).  Forward (K = false: no
// arg-min edge) and backward take the same alpha and the same decisions.
template <int WIN, bool K = true>
__device__ __forceinline__ bool frag_alpha(const TriRecord& r, double dx, double dy,
                                           float alpha_max, Frag& f)
{
    int k = 0;
    if constexpr (WIN == TS_WINDOW_SIGMOID) {
        const double d = K ? edge_min(r.A, r.B, r.C, dx, dy, k)
                           : edge_min_value(r.A, r.B, r.C, dx, dy);
        sigmoid_alpha(d, r.o, r.sigma, alpha_max, f);
        f.k = k;
        return true;
    } else if constexpr (WIN == TS_WINDOW_LSE) {
        const double u = lse_u(r.A, r.B, r.C, dx, dy, (double)r.phis, f);
        window_alpha((float)(u > 0.0 ? u : 0.0), r.o, r.sigma, alpha_max, f);
        return u > 0.0;
    } else {
        const double u = K ? edge_min(r.A, r.B, r.C, dx, dy, k)
                           : edge_min_value(r.A, r.B, r.C, dx, dy);
        // clamped after the conversion: one FP32 max instead of two FP64 ones
        window_alpha(fmaxf((float)u, 0.f), r.o, r.sigma, alpha_max, f);
        f.k = k;
        return u > 0.0;
    }
}

struct Pix {
    int w, g, i;    // wave, row, lane within the row
    int px, py;
};

__device__ __forceinline__ Pix pixel_of(int tx, int ty)
{
    Pix P;
    const int tid = threadIdx.x, lane = tid & 63;
    P.w = tid >> 6;
    P.g = lane >> 4;
    P.i = lane & 15;
    P.px = tx * kTile + (P.w & 1) * 8 + (P.g & 1) * 4 + (P.i & 3);
    P.py = ty * kTile + (P.w >> 1) * 8 + (P.g >> 1) * 4 + (P.i >> 2);
    return P;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

// Largest value over the 16 lanes of each DPP row (quad swaps, then the
// half-row and row mirrors).
__device__ __forceinline__ float row_max_f(float x)
{
    x = fmaxf(x, dpp<0xB1>(x));    // quad_perm [1,0,3,2]
    x = fmaxf(x, dpp<0x4E>(x));    // quad_perm [2,3,0,1]
    x = fmaxf(x, dpp<0x141>(x));   // row_half_mirror
    x = fmaxf(x, dpp<0x140>(x));   // row_mirror
    return x;
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------

// One tile of one view.  T_final / last may be null (forward-only serving).
struct TileJob {
    int tx, ty, W, H;
    uint32_t start, end;
    float* rgb;
    float* alpha;
    float* depth;
    float* T;
    uint32_t* last;
    uint16_t* blocks;   // per list entry: blocks where it composited (null: not kept)
    float* max_weight;  // pruning statistics (null: not kept): largest T*o per triangle,
    uint32_t* pixels;   // and pixels where it is composited
    // stored-fragment variant: per pixel the number of composited fragments,
    // their first slot, and per slot the tile-list entry, alpha and the
    // transmittance in front of the fragment
    uint32_t* fcount;
    const uint32_t* foffs;
    uint32_t* fentry;
    float* falpha;
    float* fT;
};

// FS: 0 plain forward; 1 also counts each pixel's composited fragments
// (J.fcount); 2 also stores them at J.foffs[pixel] (the stored-fragment
// variant the recompute backward is measured against).
template <int WIN, bool ST, int FS = 0>
__device__ __forceinline__ void fwd_tile(const TriRecord* __restrict__ rec,
                                         const uint32_t* __restrict__ vals, const Cfg& cfg,
                                         const TileJob& J, StageT<WIN, ST>& S)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const Pix P = pixel_of(J.tx, J.ty);
    const bool inside = P.px < J.W && P.py < J.H;
    const uint32_t start = J.start, end = J.end;

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    uint32_t last = 0;
    bool done = !inside;
    uint32_t fcnt = 0, foff = 0;
    if constexpr (FS == 2) {
        if (inside) foff = J.foffs[(int64_t)P.py * J.W + P.px];
    }

    const uint32_t my_bit = 1u << (4 * P.w + P.g);
    const double dxt = (double)(P.px - J.tx * kTile), dyt = (double)(P.py - J.ty * kTile);
    for (uint32_t b = start; b < end; b += kBatch) {
        const int n = (int)min((uint32_t)kBatch, end - b);
        __syncthreads();
        if (tid < n) {
            const uint32_t tri = vals[b + tid];
            // the statistics' max-weight word; without statistics, the blocks
            // where the entry composited (one word per entry: no shifts per step)
            S.tri[tid] = 0u;
            S.hit[tid] = (uint16_t)stage_rec<true>(S, rec, tri, J.tx * kTile, J.ty * kTile);
        }
        if (ST && tid < kBatch / 2) S.comp[tid] = 0u;
        __syncthreads();
        const Lens L = build_lists(S, n, P.w, lane, n, n, n, n);
        uint32_t* px = reinterpret_cast<uint32_t*>(S.hit);   // 16 bits per entry
        if constexpr (ST) {   // the hit words are dead once every wave has its lists
            __syncthreads();
            if (tid < kBatch / 2) px[tid] = 0u;
            __syncthreads();
        }
        // each lane walks its row's list; a row stops once all its pixels are
        // done, the wave once no row has work left
        const int len = per_row(P.g, L.n0, L.n1, L.n2, L.n3);
        const uint8_t* lst = S.list[4 * P.w + P.g];
        int jn = lst[0];                 // next entry (read one step ahead)
        bool act = !done && 0 < len;
        // the test at the bottom keeps the loop a single block (no copies
        // of the blend state per step)
        if (__ballot(act) != 0ull) for (int k = 0;;) {
            // an idle lane reads slot 0 (always staged): a stale slot could hold
            // non-finite values, and 0 * inf in the branch-free blend is NaN
            const int jl = jn;              // this step's entry of the row's list
            const int j = act ? jl : 0;
            jn = lst[k + 1 < kBatch ? k + 1 : 0];
            const TriRecord r = read_rec<true>(S, j);
            Frag f;
            const bool in = frag_alpha<WIN, false>(r, dxt, dyt, cfg.alpha_max, f);
            const bool contrib = act && in && f.a >= cfg.alpha_min;
            const float Tn = T * (1.f - f.a);
            const bool stop = contrib && Tn < cfg.T_min;
            const bool comp = contrib && !stop;
            const float wgt = comp ? f.a * T : 0.f;
            const float tw = comp ? T * r.o : 0.f;   // blending weight T*o (pruning)
            if constexpr (FS != 0) {
                if (comp) {
                    if constexpr (FS == 2) {
                        const uint32_t q = foff + fcnt;
                        J.fentry[q] = b - start + (uint32_t)j;
                        J.falpha[q] = f.a;
                        J.fT[q] = T;
                    }
                    ++fcnt;
                }
            }
            C0 = fmaf(wgt, r.rgb[0], C0);
            C1 = fmaf(wgt, r.rgb[1], C1);
            C2 = fmaf(wgt, r.rgb[2], C2);
            D = fmaf(wgt, r.z, D);
            T = comp ? Tn : T;
            last = comp ? b - start + (uint32_t)j + 1u : last;
            done = done || stop;
            if (ST || J.blocks) {
                const uint64_t cm = __ballot(comp);
                const uint32_t rowbits = (uint32_t)(cm >> (16 * P.g)) & 0xffffu;
                if (J.blocks && P.i == 0 && rowbits != 0u) {   // the entry composited in this block
                    if constexpr (ST) atomicOr(&S.comp[jl >> 1], my_bit << (16 * (jl & 1)));
                    else atomicOr(&S.tri[jl], my_bit);
                }
                if constexpr (ST) {   // pruning statistics of the row's entry, in LDS
                    const float mw = row_max_f(tw);
                    if (P.i == 0 && rowbits != 0u) {
                        atomicMax(&S.tri[jl], __float_as_uint(mw));
                        atomicAdd(&px[jl >> 1], (uint32_t)__popc(rowbits) << (16 * (jl & 1)));
                    }
                }
            }
            ++k;
            act = !done && k < len;
            if (__ballot(act) == 0ull) break;
        }
        const bool all_done = __syncthreads_and(done);
        if (J.blocks && tid < n)
            J.blocks[b + tid] = ST ? (uint16_t)(S.comp[tid >> 1] >> (16 * (tid & 1)))
                                   : (uint16_t)S.tri[tid];
        if constexpr (ST) {
            if (tid < n && S.tri[tid] != 0u) {
                const uint32_t tri = vals[b + tid];
                atomicMax(reinterpret_cast<uint32_t*>(J.max_weight) + tri, S.tri[tid]);
                atomicAdd(J.pixels + tri, (px[tid >> 1] >> (16 * (tid & 1))) & 0xffffu);
            }
        }
        if (all_done) break;
    }
    if (inside) {
        const int64_t p = (int64_t)P.py * J.W + P.px;
        const int64_t hw = (int64_t)J.W * J.H;
        J.rgb[p] = fmaf(cfg.bg[0], T, C0);
        J.rgb[hw + p] = fmaf(cfg.bg[1], T, C1);
        J.rgb[2 * hw + p] = fmaf(cfg.bg[2], T, C2);
        J.alpha[p] = 1.f - T;
        J.depth[p] = D;
        if (J.T) J.T[p] = T;
        if (J.last) J.last[p] = last;
        if constexpr (FS == 1) J.fcount[p] = fcnt;
    }
}

template <int WIN, bool ST>
__global__ __launch_bounds__(256) void k_raster_fwd(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, Cam cam, Cfg cfg,
    int tiles_x, int num_tiles, float* __restrict__ out_rgb, float* __restrict__ out_alpha,
    float* __restrict__ out_depth, float* __restrict__ out_T, uint32_t* __restrict__ out_last,
    uint16_t* __restrict__ out_blocks, float* __restrict__ max_weight,
    uint32_t* __restrict__ pixels)
{
    __shared__ StageT<WIN, ST> S;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    if ((unsigned)tile >= (unsigned)num_tiles) return;   // a corrupt order never reads past ranges
    TileJob J{tile % tiles_x, tile / tiles_x, cam.W, cam.H, ranges[2 * tile],
              ranges[2 * tile + 1], out_rgb, out_alpha, out_depth, out_T, out_last, out_blocks,
              max_weight, pixels};
    fwd_tile(rec, vals, cfg, J, S);
}

// The forward of the stored-fragment variant: FS = 1 counts the composited
// fragments of every pixel, FS = 2 stores them (see fwd_tile).
template <int WIN, int FS>
__global__ __launch_bounds__(256) void k_raster_fwd_frag(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, Cam cam, Cfg cfg,
    int tiles_x, int num_tiles, float* __restrict__ out_rgb, float* __restrict__ out_alpha,
    float* __restrict__ out_depth, float* __restrict__ out_T, uint32_t* __restrict__ out_last,
    uint16_t* __restrict__ out_blocks, FragStore fs)
{
    __shared__ StageT<WIN, false> S;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    if ((unsigned)tile >= (unsigned)num_tiles) return;
    TileJob J{tile % tiles_x, tile / tiles_x, cam.W, cam.H, ranges[2 * tile],
              ranges[2 * tile + 1], out_rgb, out_alpha, out_depth, out_T, out_last, out_blocks,
              nullptr, nullptr, fs.count, fs.offset, fs.entry, fs.alpha, fs.T};
    fwd_tile<WIN, false, FS>(rec, vals, cfg, J, S);
}

// Persistent variant over the tiles of several views: each workgroup takes
// the next tile from a queue until the batch's tiles run out.  views[] is
// sorted by tile_offset; ctl[0] = views in the batch, ctl[1] = their tiles
// (both already clamped to the buffers).
template <int WIN>
__global__ __launch_bounds__(256) void k_raster_fwd_queue(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order,
    const ts_view* __restrict__ views, const uint32_t* __restrict__ ctl, Cfg cfg,
    uint32_t* __restrict__ queue, float* __restrict__ out_rgb, float* __restrict__ out_alpha,
    float* __restrict__ out_depth)
{
    __shared__ StageT<WIN> S;
    // the queue slot lives in the stage's block-mask words of the forward
    // with statistics, which this forward never touches.  A separate
    // variable would push the workgroup past 25 LDS allocation units (four
    // per CU, not five).
    uint32_t& s_t = S.comp[0];
    const uint32_t nviews = ctl[0], total = ctl[1];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t q = s_t;
        if (q >= total) break;
        const uint32_t t = order ? order[q] : q;
        if (t >= total) continue;
        uint32_t v = 0;
        while (v + 1 < nviews && views[v + 1].tile_offset <= t) ++v;
        const ts_view& V = views[v];
        const uint32_t local = t - V.tile_offset;
        const int64_t po = (int64_t)V.pixel_offset;
        TileJob J{(int)(local % V.tiles_x), (int)(local / V.tiles_x), V.cam.width, V.cam.height,
                  ranges[2 * t], ranges[2 * t + 1], out_rgb + 3 * po, out_alpha + po,
                  out_depth + po, nullptr, nullptr, nullptr, nullptr, nullptr};
        fwd_tile(rec, vals, cfg, J, S);
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// Sum 16 per-lane values over the 16 lanes of each DPP row by
// transpose-and-add: each step pairs lanes across one bit of the lane index
// within the row (row_ror:8, row_half_mirror, quad_perm) and each lane keeps
// the half of its values its partner sends it, so the values per lane halve.
// 45 VALU, no LDS.  On return lane i of a row holds the row total of slot i.
__device__ __forceinline__ float row_reduce16(const float (&v)[16], int i)
{
    float a8[8], a4[4], a2[2];
    const bool b3 = i & 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float send = b3 ? v[k] : v[k + 8];
        const float keep = b3 ? v[k + 8] : v[k];
        a8[k] = keep + dpp<0x128>(send);           // row_ror:8      (partner i ^ 8)
    }
    const bool b2 = i & 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float send = b2 ? a8[k] : a8[k + 4];
        const float keep = b2 ? a8[k + 4] : a8[k];
        a4[k] = keep + dpp<0x141>(send);           // row_half_mirror (partner i ^ 7)
    }
    const bool b1 = i & 2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float send = b1 ? a4[k] : a4[k + 2];
        const float keep = b1 ? a4[k + 2] : a4[k];
        a2[k] = keep + dpp<0x4E>(send);            // quad_perm [2,3,0,1] (partner i ^ 2)
    }
    const bool b0 = i & 1;
    return (b0 ? a2[1] : a2[0]) + dpp<0xB1>(b0 ? a2[0] : a2[1]);   // quad_perm [1,0,3,2]
}

// Maximum over the 16 lanes of each row.
__device__ __forceinline__ uint32_t row_max(uint32_t x)
{
    x = max(x, dpp_u<0x128>(x));
    x = max(x, dpp_u<0x141>(x));
    x = max(x, dpp_u<0x4E>(x));
    x = max(x, dpp_u<0xB1>(x));
    return x;
}

// SF: the stored-fragment variant: the composited fragments of each pixel,
// their alphas and transmittances come from the forward's store (fs) instead
// of the recomputed cut-off decisions and T_before = T_after / (1 - alpha).
template <int WIN, bool SF = false>
__global__ __launch_bounds__(256) void k_raster_bwd(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, Cam cam, Cfg cfg,
    int tiles_x, int num_tiles, const float* __restrict__ dL_drgb,
    const float* __restrict__ dL_dalpha, const float* __restrict__ dL_ddepth,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last_in,
    const uint16_t* __restrict__ blocks, float* __restrict__ g2d, FragStore fs)
{
    __shared__ StageT<WIN> S;
    __shared__ uint32_t s_max;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    if ((unsigned)tile >= (unsigned)num_tiles) return;   // a corrupt order never reads past ranges
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const Pix P = pixel_of(tx, ty);
    const bool inside = P.px < cam.W && P.py < cam.H;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    const int64_t p = (int64_t)P.py * cam.W + P.px;
    const int64_t hw = (int64_t)cam.W * cam.H;
    const double dxt = (double)(P.px - tx * kTile), dyt = (double)(P.py - ty * kTile);
    float T = 1.f, Tf = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gA = 0.f, gD = 0.f;
    uint32_t my_last = 0;
    if (inside) {
        Tf = T_final[p];
        T = Tf;
        my_last = min(last_in[p], end - start);   // never beyond this tile's list
        g0 = dL_drgb[p];
        g1 = dL_drgb[hw + p];
        g2 = dL_drgb[2 * hw + p];
        gA = dL_dalpha ? dL_dalpha[p] : 0.f;
        gD = dL_ddepth ? dL_ddepth[p] : 0.f;
    }
    // stored fragments of the pixel, walked from its last one back: the next
    // one to meet (entry, alpha, T) is held in registers, its successor loaded
    // as soon as it is consumed
    int fcur = -1, flo = 0;
    uint32_t fe = 0xffffffffu;
    float fa = 0.f, fTb = 1.f;
    if constexpr (SF) {
        if (inside) {
            flo = (int)fs.offset[p];
            fcur = flo + (int)fs.count[p] - 1;
            if (fcur >= flo) {
                fe = fs.entry[fcur];
                fa = fs.alpha[fcur];
                fTb = fs.T[fcur];
            }
        }
    }
    // alpha-gradient part that multiplies T_final / (1 - a): dL/dalpha minus
    // the background seen through the remaining transmittance
    const float gT = gA - (g0 * cfg.bg[0] + g1 * cfg.bg[1] + g2 * cfg.bg[2]);
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;   // sum of w c and w z behind

    // entries each row needs: up to the last one any of its pixels composited
    const uint32_t rmax = row_max(my_last);
    const int rl0 = (int)__builtin_amdgcn_readlane(rmax, 0);
    const int rl1 = (int)__builtin_amdgcn_readlane(rmax, 16);
    const int rl2 = (int)__builtin_amdgcn_readlane(rmax, 32);
    const int rl3 = (int)__builtin_amdgcn_readlane(rmax, 48);
    if (tid == 0) s_max = 0u;
    __syncthreads();
    if (lane == 0) atomicMax(&s_max, (uint32_t)max(max(rl0, rl1), max(rl2, rl3)));
    __syncthreads();
    const uint32_t jmax = s_max;   // entries any pixel of the tile needs

    for (uint32_t hi_ = jmax; hi_ > 0;) {
        const uint32_t lo_ = hi_ > (uint32_t)kBatch ? hi_ - kBatch : 0u;
        const int n = (int)(hi_ - lo_);
        __syncthreads();
        if (tid < n) {
            const uint32_t tri = vals[start + lo_ + tid];
            S.tri[tid] = tri;
            if (blocks) {   // the forward's record of where the entry composited
                stage_copy(S, rec, tri, tx * kTile, ty * kTile);
                S.hit[tid] = blocks[start + lo_ + tid];
            } else {
                S.hit[tid] = (uint16_t)stage_rec(S, rec, tri, tx * kTile, ty * kTile);
            }
        }
        __syncthreads();
        // entries of this batch each row needs (before its last composited one)
        const Lens L = build_lists(S, n, P.w, lane, rl0 - (int)lo_, rl1 - (int)lo_,
                                   rl2 - (int)lo_, rl3 - (int)lo_);
        const int len = per_row(P.g, L.n0, L.n1, L.n2, L.n3);
        const int steps = max(max(L.n0, L.n1), max(L.n2, L.n3));
        const uint8_t* lst = S.list[4 * P.w + P.g];
        int kn = len - 1;
        int jn = lst[kn >= 0 ? kn : 0];   // next entry (read one step ahead)
        for (int st = 0; st < steps; ++st) {   // back to front along each row's list
            const int k = kn;
            const int jc = k >= 0 ? jn : 0;   // idle lanes read slot 0 (always staged)
            --kn;
            jn = lst[kn >= 0 ? kn : 0];
            const int j = k >= 0 ? jc : -1;
            const TriRecord r = read_rec(S, jc);
            const int dx = P.px - r.ax, dy = P.py - r.ay;   // anchor form of the coefficients
            Frag f;
            const bool in = frag_alpha<WIN>(r, dxt, dyt, cfg.alpha_max, f);
            bool contrib;
            float Ti;
            if constexpr (SF) {
                contrib = j >= 0 && fcur >= flo && fe == lo_ + (uint32_t)j;
                if (contrib) {
                    f.a = fa;
                    Ti = fTb;
                    --fcur;
                    if (fcur >= flo) {
                        fe = fs.entry[fcur];
                        fa = fs.alpha[fcur];
                        fTb = fs.T[fcur];
                    } else {
                        fe = 0xffffffffu;
                    }
                }
            } else {
                contrib = j >= 0 && inside && lo_ + (uint32_t)j < my_last && in &&
                          f.a >= cfg.alpha_min;
            }
            if (__ballot(contrib) == 0ull) continue;

            const float rom = __builtin_amdgcn_rcpf(1.f - f.a);
            if constexpr (!SF) Ti = T * rom;    // transmittance before this fragment
            const float wgt = contrib ? f.a * Ti : 0.f;
            float v[16];
            v[11] = g0 * wgt;
            v[12] = g1 * wgt;
            v[13] = g2 * wgt;
            v[14] = gD * wgt;
            v[15] = 0.f;
            const float ga = g0 * (r.rgb[0] * Ti - S0 * rom) + g1 * (r.rgb[1] * Ti - S1 * rom) +
                             g2 * (r.rgb[2] * Ti - S2 * rom) + gD * (r.z * Ti - SD * rom) +
                             gT * Tf * rom;
            S0 = fmaf(wgt, r.rgb[0], S0);
            S1 = fmaf(wgt, r.rgb[1], S1);
            S2 = fmaf(wgt, r.rgb[2], S2);
            SD = fmaf(wgt, r.z, SD);
            T = contrib ? Ti : T;
            const bool open = contrib && f.oI <= cfg.alpha_max;   // not clamped
            const float gI = ga * r.o;
            v[9] = open ? ga * f.I : 0.f;                                  // dL/do
            if constexpr (WIN == TS_WINDOW_LSE) {
                // u = phi_lse / phi_lse(s): dphi_lse/dd_k = -w_k (softmax weight),
                // du/dr = u / phi_lse(s) (phi_lse(s) = ln 3 - r) into slot 15
                v[10] = open ? gI * f.I * (f.lg * 0.69314718055994531f) : 0.f;  // I ln u
                const float gu = open ? gI * r.sigma * f.I * __builtin_amdgcn_rcpf(f.u) : 0.f;
                const float rp = __builtin_amdgcn_rcpf(r.phis);
                const float gphi = gu * rp;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float gd = -f.w[q] * gphi;
                    v[q] = gd * (float)dx;
                    v[3 + q] = gd * (float)dy;
                    v[6 + q] = gd;
                }
                v[15] = gu * f.u * rp;
            } else {
                float gu;
                if constexpr (WIN == TS_WINDOW_SIGMOID) {
                    // I = sigmoid(d / sigma): dI/dd = I (1 - I) / sigma,
                    // dI/dsigma = -I (1 - I) d / sigma^2
                    const float rs = __builtin_amdgcn_rcpf(r.sigma);
                    const float dI = f.I * f.Ic * rs;
                    v[10] = open ? -gI * dI * f.u * rs : 0.f;
                    gu = open ? gI * dI : 0.f;
                } else {
                    v[10] = open ? gI * f.I * (f.lg * 0.69314718055994531f) : 0.f;  // I ln u
                    gu = open ? gI * r.sigma * f.I * __builtin_amdgcn_rcpf(f.u) : 0.f;
                }
                const float a_ = gu * (float)dx, b_ = gu * (float)dy;
                v[0] = f.k == 0 ? a_ : 0.f;
                v[1] = f.k == 1 ? a_ : 0.f;
                v[2] = f.k == 2 ? a_ : 0.f;
                v[3] = f.k == 0 ? b_ : 0.f;
                v[4] = f.k == 1 ? b_ : 0.f;
                v[5] = f.k == 2 ? b_ : 0.f;
                v[6] = f.k == 0 ? gu : 0.f;
                v[7] = f.k == 1 ? gu : 0.f;
                v[8] = f.k == 2 ? gu : 0.f;
            }
            const float tot = row_reduce16(v, P.i);
            // slot 15 carries dL/dr for the LogSumExp window only
            if (j >= 0 && P.i < (WIN == TS_WINDOW_LSE ? 16 : 15) && tot != 0.f)
                unsafeAtomicAdd(g2d + (int64_t)S.tri[jc] * TS_G2D_STRIDE + P.i, tot);
        }
        hi_ = lo_;
    }
}

void launch_raster_forward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                           const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                           int num_tiles, float* rgb, float* alpha, float* depth, float* T_final,
                           uint32_t* last, uint16_t* blocks, float* max_weight, uint32_t* pixels,
                           hipStream_t stream)
{
    const TriRecord* r = reinterpret_cast<const TriRecord*>(rec);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(num_tiles), dim3(kBlock), 0, stream, r, vals, ranges, order,
                           cam, cfg, tiles_x, num_tiles, rgb, alpha, depth, T_final, last, blocks,
                           max_weight, pixels);
    };
    const bool st = max_weight != nullptr;
    switch (cfg.window) {
    case TS_WINDOW_SIGMOID:
        st ? go(k_raster_fwd<TS_WINDOW_SIGMOID, true>) : go(k_raster_fwd<TS_WINDOW_SIGMOID, false>);
        break;
    case TS_WINDOW_LSE:
        st ? go(k_raster_fwd<TS_WINDOW_LSE, true>) : go(k_raster_fwd<TS_WINDOW_LSE, false>);
        break;
    default:
        st ? go(k_raster_fwd<TS_WINDOW_PAPER, true>) : go(k_raster_fwd<TS_WINDOW_PAPER, false>);
        break;
    }
}

__global__ __launch_bounds__(256) void k_prune_views(uint32_t* __restrict__ pixels,
                                                     uint32_t* __restrict__ views, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    views[i] += pixels[i] > 1u ? 1u : 0u;
    pixels[i] = 0u;
}

void launch_prune_views(uint32_t* pixels, uint32_t* views, int64_t N, hipStream_t stream)
{
    if (N > 0)
        hipLaunchKernelGGL(k_prune_views, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream,
                           pixels, views, N);
}

void launch_raster_forward_queue(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                                 const uint32_t* order, const ts_view* views,
                                 const uint32_t* ctl, const Cfg& cfg, uint32_t* queue,
                                 int workgroups, float* rgb, float* alpha, float* depth,
                                 hipStream_t stream)
{
    const TriRecord* r = reinterpret_cast<const TriRecord*>(rec);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(workgroups), dim3(kBlock), 0, stream, r, vals, ranges,
                           order, views, ctl, cfg, queue, rgb, alpha, depth);
    };
    switch (cfg.window) {
    case TS_WINDOW_SIGMOID: go(k_raster_fwd_queue<TS_WINDOW_SIGMOID>); break;
    case TS_WINDOW_LSE: go(k_raster_fwd_queue<TS_WINDOW_LSE>); break;
    default: go(k_raster_fwd_queue<TS_WINDOW_PAPER>); break;
    }
}

void launch_raster_backward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                            const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                            int num_tiles, const float* dL_drgb, const float* dL_dalpha,
                            const float* dL_ddepth, const float* T_final,
                            const uint32_t* last, const uint16_t* blocks, float* g2d,
                            hipStream_t stream, const FragStore* fs)
{
    const TriRecord* r = reinterpret_cast<const TriRecord*>(rec);
    const FragStore none{};
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(num_tiles), dim3(kBlock), 0, stream, r, vals, ranges, order,
                           cam, cfg, tiles_x, num_tiles, dL_drgb, dL_dalpha, dL_ddepth, T_final,
                           last, blocks, g2d, fs ? *fs : none);
    };
    if (fs) {
        switch (cfg.window) {
        case TS_WINDOW_SIGMOID: go(k_raster_bwd<TS_WINDOW_SIGMOID, true>); break;
        case TS_WINDOW_LSE: go(k_raster_bwd<TS_WINDOW_LSE, true>); break;
        default: go(k_raster_bwd<TS_WINDOW_PAPER, true>); break;
        }
        return;
    }
    switch (cfg.window) {
    case TS_WINDOW_SIGMOID: go(k_raster_bwd<TS_WINDOW_SIGMOID>); break;
    case TS_WINDOW_LSE: go(k_raster_bwd<TS_WINDOW_LSE>); break;
    default: go(k_raster_bwd<TS_WINDOW_PAPER>); break;
    }
}

void launch_raster_forward_fragments(const void* rec, const uint32_t* vals,
                                     const uint32_t* ranges, const uint32_t* order,
                                     const Cam& cam, const Cfg& cfg, int tiles_x, int num_tiles,
                                     float* rgb, float* alpha, float* depth, float* T_final,
                                     uint32_t* last, uint16_t* blocks, int mode,
                                     const FragStore& fs, hipStream_t stream)
{
    const TriRecord* r = reinterpret_cast<const TriRecord*>(rec);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(num_tiles), dim3(kBlock), 0, stream, r, vals, ranges, order,
                           cam, cfg, tiles_x, num_tiles, rgb, alpha, depth, T_final, last, blocks,
                           fs);
    };
    const bool store = mode == 2;
    switch (cfg.window) {
    case TS_WINDOW_SIGMOID:
        store ? go(k_raster_fwd_frag<TS_WINDOW_SIGMOID, 2>) : go(k_raster_fwd_frag<TS_WINDOW_SIGMOID, 1>);
        break;
    case TS_WINDOW_LSE:
        store ? go(k_raster_fwd_frag<TS_WINDOW_LSE, 2>) : go(k_raster_fwd_frag<TS_WINDOW_LSE, 1>);
        break;
    default:
        store ? go(k_raster_fwd_frag<TS_WINDOW_PAPER, 2>) : go(k_raster_fwd_frag<TS_WINDOW_PAPER, 1>);
        break;
    }
}

}  // namespace ts
