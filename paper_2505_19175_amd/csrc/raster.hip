// raster.hip -- per-tile compositing on gfx950: forward (front to back) and
// backward (back to front, transmittance recovered from the final value).
//
// One 256-thread workgroup per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1), lane l the pixel (l & 7, l >> 3) of it.  The tile's list
// is walked in batches of 256 entries staged through LDS: each thread copies
// one record as seven 16-byte chunks into chunk-major arrays (consecutive
// lanes write consecutive 16-byte slots, so the staging writes are free of
// bank conflicts) and marks the quadrants the record's tight box touches.
// Each wave then visits only the entries that touch its quadrant, found by
// scalar bit scans of ballot masks, and reads each one as LDS broadcasts.
// The window is evaluated as three FP64 affine functions per pixel (gfx950
// issues v_fma_f64 at the rate of unpacked v_fma_f32); the rest is FP32,
// written without branches so a wave issues one path per entry.
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kBatch = kBlock;   // entries staged per batch
constexpr int kChunks = 7;       // 16-byte chunks of a record the raster reads

struct Stage {
    float4 q[kChunks][kBatch];
    uint8_t hit[kBatch];
};

union RecView {
    float4 q[8];
    TriRecord r;
};

__device__ __forceinline__ bool quad_hit(const TriRecord& r, int qx0, int qy0)
{
    return r.px0 <= qx0 + 7 && r.px1 >= qx0 && r.py0 <= qy0 + 7 && r.py1 >= qy0;
}

// Copy record `tri` into LDS slot threadIdx.x; return the 4-bit mask of the
// tile's 8x8 quadrants its tight box touches (bit w = quadrant of wave w).
__device__ __forceinline__ uint32_t stage_rec(Stage& S, const TriRecord* __restrict__ rec,
                                              uint32_t tri, int tx0, int ty0)
{
    const float4* src = reinterpret_cast<const float4*>(rec + tri);
    RecView u;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) u.q[c] = src[c];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) S.q[c][threadIdx.x] = u.q[c];
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        m |= quad_hit(u.r, tx0 + (w & 1) * 8, ty0 + (w >> 1) * 8) ? (1u << w) : 0u;
    return m;
}

__device__ __forceinline__ TriRecord read_rec(const Stage& S, int j)
{
    RecView u;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) u.q[c] = S.q[c][j];
    u.q[7] = make_float4(0.f, 0.f, 0.f, 0.f);
    return u.r;
}

// Entries of the current batch whose box touches wave w's quadrant: one
// 64-bit mask per 64 entries.
__device__ __forceinline__ void wave_hits(const uint8_t* s_hit, int n, int w, int lane,
                                          uint64_t (&hits)[kBatch / 64])
{
#pragma unroll
    for (int c = 0; c < kBatch / 64; ++c) {
        const int j = c * 64 + lane;
        hits[c] = __ballot(j < n && ((s_hit[j] >> w) & 1u));
    }
}

// Window and opacity of a record at pixel offset (dx, dy); u <= 0 gives
// alpha = 0.  Forward and backward call exactly this.
__device__ __forceinline__ double frag_alpha(const TriRecord& r, int dx, int dy,
                                             float alpha_max, Frag& f)
{
    int k;
    const double u = edge_min(r.A, r.B, r.C, (double)dx, (double)dy, k);
    window_alpha(u > 0.0 ? u : 0.0, r.o, r.sigma, alpha_max, f);
    f.k = k;
    return u;
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
};

__device__ __forceinline__ void fwd_tile(const TriRecord* __restrict__ rec,
                                         const uint32_t* __restrict__ vals, const Cfg& cfg,
                                         const TileJob& J, Stage& S)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int qx0 = J.tx * kTile + (w & 1) * 8, qy0 = J.ty * kTile + (w >> 1) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < J.W && py < J.H;
    const uint32_t start = J.start, end = J.end;

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    uint32_t last = 0;
    bool done = !inside;

    for (uint32_t b = start; b < end; b += kBatch) {
        const int n = (int)min((uint32_t)kBatch, end - b);
        __syncthreads();
        if (tid < n) S.hit[tid] = (uint8_t)stage_rec(S, rec, vals[b + tid], J.tx * kTile, J.ty * kTile);
        __syncthreads();
        uint64_t hits[kBatch / 64];
        wave_hits(S.hit, n, w, lane, hits);
        bool wave_done = __ballot(!done) == 0ull;
        for (int c = 0; c < kBatch / 64 && !wave_done; ++c) {
            uint64_t m = hits[c];
            while (m != 0ull) {
                const int j = c * 64 + __builtin_ctzll(m);
                m &= m - 1ull;
                const TriRecord r = read_rec(S, j);
                Frag f;
                const double u = frag_alpha(r, px - r.ax, py - r.ay, cfg.alpha_max, f);
                const bool contrib = !done && u > 0.0 && f.a >= cfg.alpha_min;
                const float Tn = T * (1.f - f.a);
                const bool stop = contrib && Tn < cfg.T_min;
                const bool comp = contrib && !stop;
                const float wgt = comp ? f.a * T : 0.f;
                C0 = fmaf(wgt, r.rgb[0], C0);
                C1 = fmaf(wgt, r.rgb[1], C1);
                C2 = fmaf(wgt, r.rgb[2], C2);
                D = fmaf(wgt, r.z, D);
                T = comp ? Tn : T;
                last = comp ? b - start + (uint32_t)j + 1u : last;
                done = done || stop;
                if (__ballot(!done) == 0ull) {
                    wave_done = true;
                    break;
                }
            }
        }
        if (__syncthreads_and(done)) break;
    }
    if (inside) {
        const int64_t p = (int64_t)py * J.W + px;
        const int64_t hw = (int64_t)J.W * J.H;
        J.rgb[p] = fmaf(cfg.bg[0], T, C0);
        J.rgb[hw + p] = fmaf(cfg.bg[1], T, C1);
        J.rgb[2 * hw + p] = fmaf(cfg.bg[2], T, C2);
        J.alpha[p] = 1.f - T;
        J.depth[p] = D;
        if (J.T) J.T[p] = T;
        if (J.last) J.last[p] = last;
    }
}

__global__ __launch_bounds__(256) void k_raster_fwd(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, Cam cam, Cfg cfg,
    int tiles_x, float* __restrict__ out_rgb, float* __restrict__ out_alpha,
    float* __restrict__ out_depth, float* __restrict__ out_T, uint32_t* __restrict__ out_last)
{
    __shared__ Stage S;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    TileJob J{tile % tiles_x, tile / tiles_x, cam.W, cam.H, ranges[2 * tile],
              ranges[2 * tile + 1], out_rgb, out_alpha, out_depth, out_T, out_last};
    fwd_tile(rec, vals, cfg, J, S);
}

// Persistent variant over the tiles of several views: each workgroup takes
// the next tile from a queue until the batch's tiles run out.  views[] is
// sorted by tile_offset; ctl[0] = views in the batch, ctl[1] = their tiles
// (both already clamped to the buffers).
__global__ __launch_bounds__(256) void k_raster_fwd_queue(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order,
    const ts_view* __restrict__ views, const uint32_t* __restrict__ ctl, Cfg cfg,
    uint32_t* __restrict__ queue, float* __restrict__ out_rgb, float* __restrict__ out_alpha,
    float* __restrict__ out_depth)
{
    __shared__ Stage S;
    __shared__ uint32_t s_t;
    const uint32_t nviews = ctl[0], total = ctl[1];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t q = s_t;
        if (q >= total) break;
        const uint32_t t = order ? order[q] : q;
        uint32_t v = 0;
        while (v + 1 < nviews && views[v + 1].tile_offset <= t) ++v;
        const ts_view& V = views[v];
        const uint32_t local = t - V.tile_offset;
        const int64_t po = (int64_t)V.pixel_offset;
        TileJob J{(int)(local % V.tiles_x), (int)(local / V.tiles_x), V.cam.width, V.cam.height,
                  ranges[2 * t], ranges[2 * t + 1], out_rgb + 3 * po, out_alpha + po,
                  out_depth + po, nullptr, nullptr};
        fwd_tile(rec, vals, cfg, J, S);
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}

// Sum 16 per-lane values over the 64 lanes of a wave by transpose-and-add:
// each step pairs lanes across one lane-index bit, and each lane keeps the
// half of its values the partner sends it, so the values per lane halve.
// Bits 5 and 4 use gfx950's v_permlane32_swap / v_permlane16_swap, bits 3
// and 2 DPP row_ror:8 / row_half_mirror, then quad DPP adds finish.  No LDS
// traffic.  On return lane L holds the total of slot L >> 2.
__device__ __forceinline__ float wave_reduce16(const float (&v)[16], int lane)
{
    float a8[8], a4[4], a2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                        __float_as_uint(v[i + 8]), false, false);
        a8[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a8[i]),
                                                        __float_as_uint(a8[i + 4]), false, false);
        a4[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    const bool b3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float send = b3 ? a4[i] : a4[i + 2];
        const float keep = b3 ? a4[i + 2] : a4[i];
        a2[i] = keep + dpp<0x128>(send);          // row_ror:8 (partner lane ^ 8)
    }
    const bool b2 = lane & 4;
    float x = (b2 ? a2[1] : a2[0]) + dpp<0x141>(b2 ? a2[0] : a2[1]);   // row_half_mirror
    x += dpp<0x4E>(x);                             // quad_perm [2,3,0,1]
    x += dpp<0xB1>(x);                             // quad_perm [1,0,3,2]
    return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d, 64));
    return x;
}

__global__ __launch_bounds__(256) void k_raster_bwd(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, Cam cam, Cfg cfg,
    int tiles_x, const float* __restrict__ dL_drgb, const float* __restrict__ dL_dalpha,
    const float* __restrict__ dL_ddepth, const float* __restrict__ T_final,
    const uint32_t* __restrict__ last_in, float* __restrict__ g2d)
{
    __shared__ Stage S;
    __shared__ uint32_t s_tri[kBatch];
    __shared__ uint32_t s_max;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int qx0 = tx * kTile + (w & 1) * 8, qy0 = ty * kTile + (w >> 1) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.W && py < cam.H;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    const int64_t p = (int64_t)py * cam.W + px;
    const int64_t hw = (int64_t)cam.W * cam.H;
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
    // alpha-gradient part that multiplies T_final / (1 - a): dL/dalpha minus
    // the background seen through the remaining transmittance
    const float gT = gA - (g0 * cfg.bg[0] + g1 * cfg.bg[1] + g2 * cfg.bg[2]);
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;   // sum of w c and w z behind
    const uint32_t wave_last = wave_max(my_last);   // entries this wave needs

    if (tid == 0) s_max = 0u;
    __syncthreads();
    if (lane == 0) atomicMax(&s_max, wave_last);
    __syncthreads();
    const uint32_t jmax = s_max;   // entries any pixel of the tile needs

    for (uint32_t hi_ = jmax; hi_ > 0;) {
        const uint32_t lo_ = hi_ > (uint32_t)kBatch ? hi_ - kBatch : 0u;
        const int n = (int)(hi_ - lo_);
        __syncthreads();
        if (tid < n) {
            const uint32_t tri = vals[start + lo_ + tid];
            s_tri[tid] = tri;
            S.hit[tid] = (uint8_t)stage_rec(S, rec, tri, tx * kTile, ty * kTile);
        }
        __syncthreads();
        uint64_t hits[kBatch / 64];
        wave_hits(S.hit, n, w, lane, hits);
        // drop entries past the last one any pixel of this wave composited
        const int lim = wave_last > lo_ ? (int)min(wave_last - lo_, (uint32_t)n) : 0;
#pragma unroll
        for (int c = 0; c < kBatch / 64; ++c) {
            const int keep = min(max(lim - c * 64, 0), 64);
            hits[c] &= keep == 64 ? ~0ull : ((1ull << keep) - 1ull);
        }
        for (int c = kBatch / 64 - 1; c >= 0; --c) {
            uint64_t m = hits[c];
            while (m != 0ull) {
                const int jj = 63 - __builtin_clzll(m);   // back to front
                m &= ~(1ull << jj);
                const int j = c * 64 + jj;
                const uint32_t idx = lo_ + (uint32_t)j;   // entry index within the tile
                const TriRecord r = read_rec(S, j);
                const int dx = px - r.ax, dy = py - r.ay;
                Frag f;
                const double u = frag_alpha(r, dx, dy, cfg.alpha_max, f);
                const bool contrib = inside && idx < my_last && u > 0.0 && f.a >= cfg.alpha_min;
                if (__ballot(contrib) == 0ull) continue;

                const float rom = __builtin_amdgcn_rcpf(1.f - f.a);
                const float Ti = T * rom;           // transmittance before this fragment
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
                v[10] = open ? gI * f.I * (f.lg * 0.69314718055994531f) : 0.f;  // I ln u
                const float gu = open ? gI * r.sigma * f.I * __builtin_amdgcn_rcpf(f.u) : 0.f;
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
                const float tot = wave_reduce16(v, lane);
                if ((lane & 3) == 0 && (lane >> 2) < 15 && tot != 0.f)
                    unsafeAtomicAdd(g2d + (int64_t)s_tri[j] * TS_G2D_STRIDE + (lane >> 2), tot);
            }
        }
        hi_ = lo_;
    }
}

void launch_raster_forward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                           const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                           int num_tiles, float* rgb, float* alpha, float* depth, float* T_final,
                           uint32_t* last, hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_fwd, dim3(num_tiles), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, order, cam, cfg,
                       tiles_x, rgb, alpha, depth, T_final, last);
}

void launch_raster_forward_queue(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                                 const uint32_t* order, const ts_view* views,
                                 const uint32_t* ctl, const Cfg& cfg, uint32_t* queue,
                                 int workgroups, float* rgb, float* alpha, float* depth,
                                 hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_fwd_queue, dim3(workgroups), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, order, views, ctl,
                       cfg, queue, rgb, alpha, depth);
}

void launch_raster_backward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                            const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                            int num_tiles, const float* dL_drgb, const float* dL_dalpha,
                            const float* dL_ddepth, const float* T_final,
                            const uint32_t* last, float* g2d, hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_bwd, dim3(num_tiles), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, order, cam, cfg,
                       tiles_x, dL_drgb, dL_dalpha, dL_ddepth, T_final, last, g2d);
}

}  // namespace ts
