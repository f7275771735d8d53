// raster.hip -- per-tile compositing on gfx950: forward (front to back) and
// backward (back to front, transmittance recovered from the final value).
//
// One 256-thread workgroup per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1), lane l the pixel (l & 7, l >> 3) of it.  The tile's list
// is walked in batches of 256 records staged through LDS (each thread copies
// one 128-byte record); every wave then reads the records as broadcasts.
// A record whose tight box misses a wave's quadrant is skipped by that wave
// as a whole.  The window is evaluated as three FP64 affine functions per
// pixel (gfx950 issues v_fma_f64 at the rate of unpacked v_fma_f32), the
// rest in FP32.
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kBatch = kBlock;

__device__ __forceinline__ bool quad_hit(const TriRecord& r, int qx0, int qy0)
{
    return r.px0 <= qx0 + 7 && r.px1 >= qx0 && r.py0 <= qy0 + 7 && r.py1 >= qy0;
}

// Copy one record into LDS slot threadIdx.x and return the 4-bit mask of
// the tile's 8x8 quadrants its tight box touches (bit w = quadrant of wave w).
__device__ __forceinline__ uint32_t stage(TriRecord* s_rec, const TriRecord* __restrict__ rec,
                                          uint32_t tri, int tx0, int ty0)
{
    const float4* src = reinterpret_cast<const float4*>(rec + tri);
    float4* dst = reinterpret_cast<float4*>(s_rec + threadIdx.x);
    float4 t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = src[j];
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[j] = t[j];
    const TriRecord& r = *reinterpret_cast<const TriRecord*>(t);
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        m |= quad_hit(r, tx0 + (w & 1) * 8, ty0 + (w >> 1) * 8) ? (1u << w) : 0u;
    return m;
}

// Entries of the current batch whose box touches wave w's quadrant: one
// 64-bit mask per 64 entries, from the per-entry masks written at staging.
__device__ __forceinline__ void wave_hits(const uint8_t* s_hit, int n, int w, int lane,
                                          uint64_t (&hits)[kBatch / 64])
{
#pragma unroll
    for (int c = 0; c < kBatch / 64; ++c) {
        const int j = c * 64 + lane;
        hits[c] = __ballot(j < n && ((s_hit[j] >> w) & 1u));
    }
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
                                         const TileJob& J, TriRecord* s_rec, uint8_t* s_hit)
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
        if (tid < n)
            s_hit[tid] = (uint8_t)stage(s_rec, rec, vals[b + tid], J.tx * kTile, J.ty * kTile);
        __syncthreads();
        uint64_t hits[kBatch / 64];
        wave_hits(s_hit, n, w, lane, hits);
        bool wave_done = __ballot(!done) == 0ull;
        for (int c = 0; c < kBatch / 64 && !wave_done; ++c) {
            uint64_t m = hits[c];
            while (m != 0ull) {
                const int j = c * 64 + __builtin_ctzll(m);
                m &= m - 1ull;
                const TriRecord& r = s_rec[j];
                if (!done) {
                    int k;
                    const double u = edge_min(r.A, r.B, r.C, (double)(px - r.ax),
                                              (double)(py - r.ay), k);
                    if (u > 0.0) {
                        Frag f;
                        window_alpha(u, r.o, r.sigma, cfg.alpha_max, f);
                        if (f.a >= cfg.alpha_min) {
                            const float Tn = T * (1.f - f.a);
                            if (Tn < cfg.T_min) {
                                done = true;
                            } else {
                                const float wgt = f.a * T;
                                C0 = fmaf(wgt, r.rgb[0], C0);
                                C1 = fmaf(wgt, r.rgb[1], C1);
                                C2 = fmaf(wgt, r.rgb[2], C2);
                                D = fmaf(wgt, r.z, D);
                                T = Tn;
                                last = b - start + (uint32_t)j + 1u;
                            }
                        }
                    }
                }
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
    const uint32_t* __restrict__ ranges, Cam cam, Cfg cfg, int tiles_x,
    float* __restrict__ out_rgb, float* __restrict__ out_alpha, float* __restrict__ out_depth,
    float* __restrict__ out_T, uint32_t* __restrict__ out_last)
{
    __shared__ TriRecord s_rec[kBatch];
    __shared__ uint8_t s_hit[kBatch];
    const int tile = blockIdx.x;
    TileJob J{tile % tiles_x, tile / tiles_x, cam.W, cam.H, ranges[2 * tile],
              ranges[2 * tile + 1], out_rgb, out_alpha, out_depth, out_T, out_last};
    fwd_tile(rec, vals, cfg, J, s_rec, s_hit);
}

// Persistent variant over the tiles of several views: each workgroup takes
// the next tile from a queue until the batch's tiles run out.  views[] is
// sorted by tile_offset; ctl[0] = views in the batch, ctl[1] = their tiles.
__global__ __launch_bounds__(256) void k_raster_fwd_queue(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const ts_view* __restrict__ views,
    const uint32_t* __restrict__ ctl, Cfg cfg, uint32_t* __restrict__ queue,
    float* __restrict__ out_rgb, float* __restrict__ out_alpha, float* __restrict__ out_depth)
{
    __shared__ TriRecord s_rec[kBatch];
    __shared__ uint8_t s_hit[kBatch];
    __shared__ uint32_t s_t;
    const uint32_t nviews = ctl[0], total = ctl[1];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t t = s_t;
        if (t >= total) break;
        uint32_t v = 0;
        while (v + 1 < nviews && views[v + 1].tile_offset <= t) ++v;
        const ts_view& V = views[v];
        const uint32_t local = t - V.tile_offset;
        const int64_t po = (int64_t)V.pixel_offset;
        TileJob J{(int)(local % V.tiles_x), (int)(local / V.tiles_x), V.cam.width, V.cam.height,
                  ranges[2 * t], ranges[2 * t + 1], out_rgb + 3 * po, out_alpha + po,
                  out_depth + po, nullptr, nullptr};
        fwd_tile(rec, vals, cfg, J, s_rec, s_hit);
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// Sum 16 per-lane values over the 64 lanes of a wave.  Each exchange step
// halves the values a lane keeps (transpose-and-add), so 17 cross-lane moves
// replace 16 x 6.  On return lane L holds the total of slot L >> 2.
__device__ __forceinline__ float wave_reduce16(float (&v)[16], int lane)
{
    float a8[8], a4[4], a2[2];
    {
        const bool hi = lane & 32;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float send = hi ? v[i] : v[i + 8];
            const float keep = hi ? v[i + 8] : v[i];
            a8[i] = keep + __shfl_xor(send, 32, 64);
        }
    }
    {
        const bool hi = lane & 16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float send = hi ? a8[i] : a8[i + 4];
            const float keep = hi ? a8[i + 4] : a8[i];
            a4[i] = keep + __shfl_xor(send, 16, 64);
        }
    }
    {
        const bool hi = lane & 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float send = hi ? a4[i] : a4[i + 2];
            const float keep = hi ? a4[i + 2] : a4[i];
            a2[i] = keep + __shfl_xor(send, 8, 64);
        }
    }
    const bool hi = lane & 4;
    float x = (hi ? a2[1] : a2[0]) + __shfl_xor(hi ? a2[0] : a2[1], 4, 64);
    x += __shfl_xor(x, 2, 64);
    x += __shfl_xor(x, 1, 64);
    return x;
}

__global__ __launch_bounds__(256) void k_raster_bwd(
    const TriRecord* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, Cam cam, Cfg cfg, int tiles_x,
    const float* __restrict__ dL_drgb, const float* __restrict__ dL_dalpha,
    const float* __restrict__ dL_ddepth, const float* __restrict__ T_final,
    const uint32_t* __restrict__ last_in, float* __restrict__ g2d)
{
    __shared__ TriRecord s_rec[kBatch];
    __shared__ uint32_t s_tri[kBatch];
    __shared__ uint8_t s_hit[kBatch];
    __shared__ uint32_t s_max;
    const int tile = blockIdx.x;
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

    if (tid == 0) s_max = 0u;
    __syncthreads();
    atomicMax(&s_max, my_last);
    __syncthreads();
    const uint32_t jmax = s_max;   // list entries any pixel of the tile needs

    for (uint32_t hi_ = jmax; hi_ > 0;) {
        const uint32_t lo_ = hi_ > (uint32_t)kBatch ? hi_ - kBatch : 0u;
        const int n = (int)(hi_ - lo_);
        __syncthreads();
        if (tid < n) {
            const uint32_t tri = vals[start + lo_ + tid];
            s_tri[tid] = tri;
            s_hit[tid] = (uint8_t)stage(s_rec, rec, tri, tx * kTile, ty * kTile);
        }
        __syncthreads();
        uint64_t hits[kBatch / 64];
        wave_hits(s_hit, n, w, lane, hits);
        for (int c = kBatch / 64 - 1; c >= 0; --c) {
          uint64_t m = hits[c];
          while (m != 0ull) {
            const int j = c * 64 + 63 - __builtin_clzll(m);   // back to front
            m &= ~(1ull << (j - c * 64));
            const uint32_t idx = lo_ + (uint32_t)j;   // entry index within the tile
            const TriRecord& r = s_rec[j];
            bool contrib = false;
            float v[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = 0.f;
            if (inside && idx < my_last) {
                const float dxf = (float)(px - r.ax), dyf = (float)(py - r.ay);
                int k;
                const double u = edge_min(r.A, r.B, r.C, (double)(px - r.ax), (double)(py - r.ay), k);
                if (u > 0.0) {
                    Frag f;
                    window_alpha(u, r.o, r.sigma, cfg.alpha_max, f);
                    if (f.a >= cfg.alpha_min) {
                        contrib = true;
                        const float om = 1.f - f.a;
                        const float rom = __builtin_amdgcn_rcpf(om);
                        const float Ti = T * rom;          // transmittance before this fragment
                        const float wgt = f.a * Ti;
                        v[11] = g0 * wgt;
                        v[12] = g1 * wgt;
                        v[13] = g2 * wgt;
                        v[14] = gD * wgt;
                        float ga = g0 * (r.rgb[0] * Ti - S0 * rom) + g1 * (r.rgb[1] * Ti - S1 * rom) +
                                   g2 * (r.rgb[2] * Ti - S2 * rom) + gD * (r.z * Ti - SD * rom) +
                                   gT * Tf * rom;
                        S0 = fmaf(wgt, r.rgb[0], S0);
                        S1 = fmaf(wgt, r.rgb[1], S1);
                        S2 = fmaf(wgt, r.rgb[2], S2);
                        SD = fmaf(wgt, r.z, SD);
                        T = Ti;
                        if (f.oI <= cfg.alpha_max) {       // not clamped
                            v[9] = ga * f.I;                         // dL/do
                            const float gI = ga * r.o;
                            v[10] = gI * f.I * (f.lg * 0.69314718055994531f);  // dI/dsigma = I ln u
                            const float gu = gI * r.sigma * f.I * __builtin_amdgcn_rcpf(f.u);
                            const float a_ = gu * dxf, b_ = gu * dyf;
                            v[0] = k == 0 ? a_ : 0.f;
                            v[1] = k == 1 ? a_ : 0.f;
                            v[2] = k == 2 ? a_ : 0.f;
                            v[3] = k == 0 ? b_ : 0.f;
                            v[4] = k == 1 ? b_ : 0.f;
                            v[5] = k == 2 ? b_ : 0.f;
                            v[6] = k == 0 ? gu : 0.f;
                            v[7] = k == 1 ? gu : 0.f;
                            v[8] = k == 2 ? gu : 0.f;
                        }
                    }
                }
            }
            if (__ballot(contrib) != 0ull) {
                const float tot = wave_reduce16(v, lane);
                if ((lane & 3) == 0 && (lane >> 2) < 15)
                    unsafeAtomicAdd(g2d + (int64_t)s_tri[j] * TS_G2D_STRIDE + (lane >> 2), tot);
            }
          }
        }
        hi_ = lo_;
    }
}

void launch_raster_forward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                           const Cam& cam, const Cfg& cfg, int tiles_x, int num_tiles,
                           float* rgb, float* alpha, float* depth, float* T_final,
                           uint32_t* last, hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_fwd, dim3(num_tiles), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, cam, cfg, tiles_x,
                       rgb, alpha, depth, T_final, last);
}

void launch_raster_forward_queue(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                                 const ts_view* views, const uint32_t* ctl, const Cfg& cfg,
                                 uint32_t* queue, int workgroups, float* rgb, float* alpha,
                                 float* depth, hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_fwd_queue, dim3(workgroups), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, views, ctl, cfg,
                       queue, rgb, alpha, depth);
}

void launch_raster_backward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                            const Cam& cam, const Cfg& cfg, int tiles_x, int num_tiles,
                            const float* dL_drgb, const float* dL_dalpha,
                            const float* dL_ddepth, const float* T_final,
                            const uint32_t* last, float* g2d, hipStream_t stream)
{
    hipLaunchKernelGGL(k_raster_bwd, dim3(num_tiles), dim3(kBlock), 0, stream,
                       reinterpret_cast<const TriRecord*>(rec), vals, ranges, cam, cfg, tiles_x,
                       dL_drgb, dL_dalpha, dL_ddepth, T_final, last, g2d);
}

}  // namespace ts
