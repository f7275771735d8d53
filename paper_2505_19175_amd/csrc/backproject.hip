// backproject.hip -- the chain from the per-triangle 2D gradients to the
// triangle parameters (backward), and the same chain with the training
// step's Adam update applied in place.  One thread per triangle; geometry in
// FP64.
#include "adam.h"
#include "geometry.h"
#include "ts_kernels.h"

namespace ts {

// Streaming stores for the gradient arrays: they are written once per step
// and read by nothing later in the step, so they are marked non-temporal and
// do not push the soup's parameters (which the next projection reads again)
// out of the caches.  Measured: backward projection 0.234 -> 0.220 ms and
// the following projection 0.214 -> 0.180 ms on the 3M-triangle view.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_stream(float4* p, float a, float b, float c, float d)
{
    const f32x4 t = {a, b, c, d};
    __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p));
}

__device__ __forceinline__ void store_stream(float* p, float a)
{
    __builtin_nontemporal_store(a, p);
}

// Stores n floats of LDS to contiguous global memory, one 16-byte vector per
// lane where the block is full (n % 4 == 0 and 16-byte aligned), streaming.
__device__ __forceinline__ void block_store(float* __restrict__ dst, const float* src, int n)
{
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
        float4* d4 = reinterpret_cast<float4*>(dst);
        for (int f = threadIdx.x; f < n / 4; f += blockDim.x)
            store_stream(d4 + f, src[4 * f], src[4 * f + 1], src[4 * f + 2], src[4 * f + 3]);
    } else {
        for (int f = threadIdx.x; f < n; f += blockDim.x) store_stream(dst + f, src[f]);
    }
}

__device__ __forceinline__ bool aligned16(const float* a, const float* b, const float* c)
{
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
             reinterpret_cast<uintptr_t>(c)) & 15u) == 0;
}

// ---------------------------------------------------------------------------
// Backward: 2D accumulators -> window coefficients -> projected vertices ->
// camera space -> world vertices; colour -> SH coefficients and view
// direction.  Consumes g2d (re-zeroes it).
// g2d slots: 0-2 dL/dA_k, 3-5 dL/dB_k, 6-8 dL/dC_k, 9 dL/do, 10 dL/dsigma,
//            11-13 dL/drgb, 14 dL/dz, 15 dL/dr (LogSumExp window: the
//            inradius through phi_lse(s) = ln 3 - r).
// ---------------------------------------------------------------------------

// The chain of one visible triangle: its 2D accumulators (re-zeroed) ->
// window coefficients -> projected vertices -> camera space -> world
// vertices; colour -> view direction.  Outputs dL/dv (gvo), the SH basis at
// the view direction (yo; dL/dsh = yo x go3), dL/drgb where the colour is not
// clamped (go3), dL/do (go_) and dL/dsigma (gs_).
template <int DEG, int WIN>
__device__ __forceinline__ void chain_triangle(const float vv[9], int64_t i,
                                               const float4* __restrict__ cgrad, const Cam& cam,
                                               const Cfg& cfg, const short4* __restrict__ rect,
                                               float4* __restrict__ g2d, float gvo[9],
                                               float yo[(DEG + 1) * (DEG + 1)], float go3[3],
                                               float& go_, float& gs_)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    float G[16];
    {
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 t = g2d[4 * i + j];
            G[4 * j + 0] = t.x; G[4 * j + 1] = t.y; G[4 * j + 2] = t.z; G[4 * j + 3] = t.w;
            g2d[4 * i + j] = z4;
        }
    }
    go_ = G[9];
    gs_ = G[10];

    Geo g;
    project_geo(vv, cam, cfg.z_near, g);
    const short4 rc = rect[i];
    const double ax = (double)rc.x, ay = (double)rc.z;

    // coefficients -> (w_k, e_k, q_k); w_k = P / (S l_k) for Eq. 1,
    // sgn(S) / l_k for the distance form of the alternatives
    double gq[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    double ge[3][2];
    double gP = 0.0, gS = 0.0, gl[3];
    const double sgn = g.S > 0.0 ? 1.0 : -1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double w = WIN == TS_WINDOW_PAPER ? g.P / (g.S * g.len[k]) : sgn / g.len[k];
        const double qx = g.q[k][0] - ax, qy = g.q[k][1] - ay;
        const double ex = g.e[k][0], ey = g.e[k][1];
        const double gA = G[k], gB = G[3 + k], gC = G[6 + k];
        const double ck = ex * (0.5 - qy) - ey * (0.5 - qx);
        const double gw = -gA * ey + gB * ex + gC * ck;
        ge[k][0] = gB * w + gC * w * (0.5 - qy);
        ge[k][1] = -gA * w - gC * w * (0.5 - qx);
        gq[k][0] += gC * w * ey;
        gq[k][1] += -gC * w * ex;
        if constexpr (WIN == TS_WINDOW_PAPER) {   // w = P / (S l_k)
            gP += gw / (g.S * g.len[k]);
            gS += -gw * w / g.S;
        }
        gl[k] = -gw * w / g.len[k];
    }
    if constexpr (WIN == TS_WINDOW_LSE) {   // r = |S| / P
        const double gr = (double)G[15];
        gS += gr * sgn / g.P;
        gP += -gr * (fabs(g.S) / g.P) / g.P;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double gl_k = gl[k] + gP;               // P = sum l_k
        ge[k][0] += gl_k * g.e[k][0] / g.len[k];      // l_k = |e_k|
        ge[k][1] += gl_k * g.e[k][1] / g.len[k];
    }
    // S = x0 (y1 - y2) + x1 (y2 - y0) + x2 (y0 - y1)
    gq[0][0] += gS * (g.q[1][1] - g.q[2][1]);
    gq[0][1] += gS * (g.q[2][0] - g.q[1][0]);
    gq[1][0] += gS * (g.q[2][1] - g.q[0][1]);
    gq[1][1] += gS * (g.q[0][0] - g.q[2][0]);
    gq[2][0] += gS * (g.q[0][1] - g.q[1][1]);
    gq[2][1] += gS * (g.q[1][0] - g.q[0][0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {                     // e_k = q_{k+1} - q_k
        const int k1 = k == 2 ? 0 : k + 1;
        gq[k1][0] += ge[k][0]; gq[k1][1] += ge[k][1];
        gq[k][0] -= ge[k][0];  gq[k][1] -= ge[k][1];
    }

    // projection q = (fx x/z + cx, fy y/z + cy); depth key = mean z
    const double gz3 = (double)G[14] * (1.0 / 3.0);
    double gw_[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double x = g.xc[j][0], y = g.xc[j][1], z = g.xc[j][2];
        const double iz = 1.0 / z;
        const double gx0 = cam.fx * iz * gq[j][0];
        const double gx1 = cam.fy * iz * gq[j][1];
        const double gx2 = -(cam.fx * x * gq[j][0] + cam.fy * y * gq[j][1]) * iz * iz + gz3;
#pragma unroll
        for (int b = 0; b < 3; ++b)                   // R^T gx
            gw_[j][b] = (double)cam.R[b] * gx0 + (double)cam.R[3 + b] * gx1 +
                        (double)cam.R[6 + b] * gx2;
    }

    // colour: rgb = max(0, sum_k sh_k Y_k(d) + 1/2).  The projection kept
    // the unclamped channels and J[c][b] = sum_k sh_kc dY_k/d dir_b.
    double d[3], nrm;
    view_dir(vv, cam, d, nrm);
    float Y[16];
    sh_basis(DEG, (float)d[0], (float)d[1], (float)d[2], Y);
    const float4 c0 = cgrad[3 * i], c1 = cgrad[3 * i + 1], c2 = cgrad[3 * i + 2];
    const uint32_t open = __float_as_uint(c2.y);
    const float gr0 = (open & 1u) ? G[11] : 0.f;
    const float gr1 = (open & 2u) ? G[12] : 0.f;
    const float gr2 = (open & 4u) ? G[13] : 0.f;
    go3[0] = gr0; go3[1] = gr1; go3[2] = gr2;
#pragma unroll
    for (int k = 0; k < K; ++k) yo[k] = Y[k];
    float gd[3];
    gd[0] = gr0 * c0.x + gr1 * c0.w + gr2 * c1.z;
    gd[1] = gr0 * c0.y + gr1 * c1.x + gr2 * c1.w;
    gd[2] = gr0 * c0.z + gr1 * c1.y + gr2 * c2.x;
    // d = dv/|dv|, dv = centroid - camera centre, centroid = mean of vertices
    const double dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double gdv = ((double)gd[b] - d[b] * dd) / nrm * (1.0 / 3.0);
#pragma unroll
        for (int j = 0; j < 3; ++j) gw_[j][b] += gdv;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int b = 0; b < 3; ++b) gvo[3 * j + b] = (float)gw_[j][b];
}

// A block handles 256 consecutive triangles and writes their gradient rows
// through LDS, so every store of the block is contiguous (the SH gradient is
// the largest array the step writes: 12 (deg+1)^2 bytes per triangle).
template <int DEG, int WIN>
__global__ __launch_bounds__(256) void k_backproject(
    const float* __restrict__ v, const float4* __restrict__ cgrad, int64_t N, Cam cam, Cfg cfg,
    const short4* __restrict__ rect, const uint32_t* __restrict__ ntiles,
    float4* __restrict__ g2d, float* __restrict__ gv, float* __restrict__ go,
    float* __restrict__ gsig, float* __restrict__ gsh)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int NSH = 3 * K;
    __shared__ float s_gv[256 * 9];
    // SH basis at the view direction, rows padded to an odd stride so the
    // per-lane row writes hit distinct LDS banks
    constexpr int KP = K | 1;
    __shared__ float s_y[256 * KP];
    __shared__ float s_g[256 * 3];     // dL/drgb where the colour is not clamped
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 256;
    const int64_t i = base + tid;
    const int nt = (int)min((int64_t)256, N - base);

    float gvo[9], yo[K], go3[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 9; ++a) gvo[a] = 0.f;
#pragma unroll
    for (int a = 0; a < K; ++a) yo[a] = 0.f;
    float go_ = 0.f, gs_ = 0.f;

    if (i < N && ntiles[i] != 0u) {
        float vv[9];
        load_vertices(v, i, vv);
        chain_triangle<DEG, WIN>(vv, i, cgrad, cam, cfg, rect, g2d, gvo, yo, go3, go_, gs_);
    }
    if (i < N) {
        store_stream(go + i, go_);
        store_stream(gsig + i, gs_);
    }

#pragma unroll
    for (int a = 0; a < 9; ++a) s_gv[tid * 9 + a] = gvo[a];
#pragma unroll
    for (int a = 0; a < K; ++a) s_y[tid * KP + a] = yo[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) s_g[tid * 3 + a] = go3[a];
    __syncthreads();
    block_store(gv + base * 9, s_gv, nt * 9);
    // dL/dsh[t][k][c] = Y_k(d_t) dL/drgb_c, written as contiguous rows
    float* dst = gsh + base * NSH;
    const int n = nt * NSH;
    if constexpr (NSH % 4 == 0) {
        constexpr int R4 = NSH / 4;   // float4 per row
        float4* d4 = reinterpret_cast<float4*>(dst);
        if ((reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
            for (int f = tid; f < n / 4; f += 256) {
                const int t = f / R4, q0 = 4 * (f - t * R4);
                float x[4];
#pragma unroll
                for (int cq = 0; cq < 4; ++cq) {
                    const int q = q0 + cq, k = q / 3, ch = q - 3 * k;
                    x[cq] = s_y[t * KP + k] * s_g[t * 3 + ch];
                }
                store_stream(d4 + f, x[0], x[1], x[2], x[3]);
            }
            return;
        }
    }
    for (int f = tid; f < n; f += 256) {
        const int t = f / NSH, q = f - t * NSH, k = q / 3, ch = q - 3 * k;
        store_stream(dst + f, s_y[t * KP + k] * s_g[t * 3 + ch]);
    }
}

template <int DEG, int WIN>
struct BackprojectLaunch {
    static void run(dim3 grid, hipStream_t stream, const float* v, const float4* cg, int64_t N,
                    const Cam& cam, const Cfg& cfg, const short4* r4, const uint32_t* ntiles,
                    float4* g4, float* gv, float* go, float* gsig, float* gsh)
    {
        hipLaunchKernelGGL((k_backproject<DEG, WIN>), grid, dim3(256), 0, stream, v, cg, N, cam,
                           cfg, r4, ntiles, g4, gv, go, gsig, gsh);
    }
};

void launch_backproject(const float* v, const float* cgrad, int64_t N, const Cam& cam,
                        const Cfg& cfg, const int16_t* rect, const uint32_t* ntiles, float* g2d,
                        float* gv, float* go, float* gsig, float* gsh, hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256));
    dispatch_deg_win<BackprojectLaunch>(cfg.deg, cfg.window, grid, stream, v,
                                        reinterpret_cast<const float4*>(cgrad), N, cam, cfg,
                                        reinterpret_cast<const short4*>(rect), ntiles,
                                        reinterpret_cast<float4*>(g2d), gv, go, gsig, gsh);
}

// The same chain followed by the optimizer step, for training: triangles
// share no parameters, so a triangle's gradient is complete here and Adam
// runs on it at once; the gradient arrays are never written or read.  The
// block stages its vertex rows in LDS (the chain and the size loss read
// them), then updates vertices, opacity and sigma logits and SH coefficients
// element-wise over its own 256 triangles, so every access is coalesced and
// no block touches another's parameters.
struct AdamArgs {
    float* a;       // opacity logits; o = sigmoid(a)
    float* b;       // log sigma; sigma = exp(b)
    float* sh;
    float* o;       // activated copies: read (old), rewritten (new)
    float* sigma;
    float *m_v, *s_v, *m_a, *s_a, *m_b, *s_b, *m_sh, *s_sh;
    float lr_v, lr_a, lr_b, lr_dc, lr_rest;
    float add_o;    // the opacity loss's dL/do = beta_o / N
    float beta_s;
    AdamK k;
};

template <int DEG, int WIN>
__global__ __launch_bounds__(256) void k_backproject_adam(
    float* __restrict__ v, const float4* __restrict__ cgrad, int64_t N, Cam cam, Cfg cfg,
    const short4* __restrict__ rect, const uint32_t* __restrict__ ntiles,
    float4* __restrict__ g2d, AdamArgs A)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int NSH = 3 * K;
    __shared__ float s_v[256 * 9];     // vertex rows before the step
    __shared__ float s_gv[256 * 9];
    constexpr int KP = K | 1;         // odd row stride: conflict-free row writes
    __shared__ float s_y[256 * KP];
    __shared__ float s_g[256 * 3];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 256;
    const int64_t i = base + tid;
    const int nt = (int)min((int64_t)256, N - base);
    const int64_t off = 9 * base;
    for (int f = tid; f < 9 * nt; f += 256) s_v[f] = v[off + f];
    __syncthreads();

    float gvo[9], yo[K], go3[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 9; ++a) gvo[a] = 0.f;
#pragma unroll
    for (int a = 0; a < K; ++a) yo[a] = 0.f;
    float go_ = 0.f, gs_ = 0.f;
    if (i < N && ntiles[i] != 0u) {
        float vv[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) vv[a] = s_v[9 * tid + a];
        chain_triangle<DEG, WIN>(vv, i, cgrad, cam, cfg, rect, g2d, gvo, yo, go3, go_, gs_);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) s_gv[tid * 9 + a] = gvo[a];
#pragma unroll
    for (int a = 0; a < K; ++a) s_y[tid * KP + a] = yo[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) s_g[tid * 3 + a] = go3[a];
    if (tid < nt && A.beta_s != 0.f) size_loss_grad(s_v + 9 * tid, s_gv + 9 * tid, A.beta_s, N);

    // opacity and sigma logits: one element per thread
    if (i < N) {
        float m = A.m_a[i], sq = A.s_a[i];
        float p = adam_update(A.a[i], act_grad(go_, 1, A.add_o, A.o[i]), m, sq,
                              A.lr_a, A.k);
        A.m_a[i] = m; A.s_a[i] = sq; A.a[i] = p; A.o[i] = act_value(p, 1);
        m = A.m_b[i]; sq = A.s_b[i];
        p = adam_update(A.b[i], act_grad(gs_, 2, 0.f, A.sigma[i]), m, sq, A.lr_b, A.k);
        A.m_b[i] = m; A.s_b[i] = sq; A.b[i] = p; A.sigma[i] = act_value(p, 2);
    }
    __syncthreads();
    // The updates stream three arrays in and out at this kernel's low
    // occupancy (the chain's registers), so each lane moves 16-byte vectors
    // where the span allows (always for full blocks and SH degree >= 1).
    const int nv = 9 * nt;
    if ((nv & 3) == 0 && aligned16(v + off, A.m_v + off, A.s_v + off)) {
        float4* V4 = reinterpret_cast<float4*>(v + off);
        float4* M4 = reinterpret_cast<float4*>(A.m_v + off);
        float4* S4 = reinterpret_cast<float4*>(A.s_v + off);
        for (int f = tid; f < nv / 4; f += 256) {
            float4 m = M4[f], sq = S4[f], r;
            const int e = 4 * f;
            r.x = adam_update(s_v[e + 0], s_gv[e + 0], m.x, sq.x, A.lr_v, A.k);
            r.y = adam_update(s_v[e + 1], s_gv[e + 1], m.y, sq.y, A.lr_v, A.k);
            r.z = adam_update(s_v[e + 2], s_gv[e + 2], m.z, sq.z, A.lr_v, A.k);
            r.w = adam_update(s_v[e + 3], s_gv[e + 3], m.w, sq.w, A.lr_v, A.k);
            V4[f] = r; M4[f] = m; S4[f] = sq;
        }
    } else {
        for (int f = tid; f < nv; f += 256) {
            float m = A.m_v[off + f], sq = A.s_v[off + f];
            v[off + f] = adam_update(s_v[f], s_gv[f], m, sq, A.lr_v, A.k);
            A.m_v[off + f] = m;
            A.s_v[off + f] = sq;
        }
    }
    // SH: dL/dsh[t][k][c] = Y_k(d_t) dL/drgb_c; degree-0 coefficients
    // (the first three of a row) take lr_dc
    const int64_t soff = base * NSH;
    const int ns = nt * NSH;
    auto sh_grad = [&](int e, float& lr) {
        const int t = e / NSH, q = e - t * NSH, kk = q / 3, ch = q - 3 * kk;
        lr = q < 3 ? A.lr_dc : A.lr_rest;
        return s_y[t * KP + kk] * s_g[t * 3 + ch];
    };
    if ((NSH & 3) == 0 && aligned16(A.sh + soff, A.m_sh + soff, A.s_sh + soff)) {
        float4* P4 = reinterpret_cast<float4*>(A.sh + soff);
        float4* M4 = reinterpret_cast<float4*>(A.m_sh + soff);
        float4* S4 = reinterpret_cast<float4*>(A.s_sh + soff);
        for (int f = tid; f < ns / 4; f += 256) {
            float4 p = P4[f], m = M4[f], sq = S4[f];
            const int e = 4 * f;
            float lr;
            float g = sh_grad(e + 0, lr);
            p.x = adam_update(p.x, g, m.x, sq.x, lr, A.k);
            g = sh_grad(e + 1, lr);
            p.y = adam_update(p.y, g, m.y, sq.y, lr, A.k);
            g = sh_grad(e + 2, lr);
            p.z = adam_update(p.z, g, m.z, sq.z, lr, A.k);
            g = sh_grad(e + 3, lr);
            p.w = adam_update(p.w, g, m.w, sq.w, lr, A.k);
            P4[f] = p; M4[f] = m; S4[f] = sq;
        }
    } else {
        for (int f = tid; f < ns; f += 256) {
            float lr;
            const float g = sh_grad(f, lr);
            float m = A.m_sh[soff + f], sq = A.s_sh[soff + f];
            A.sh[soff + f] = adam_update(A.sh[soff + f], g, m, sq, lr, A.k);
            A.m_sh[soff + f] = m;
            A.s_sh[soff + f] = sq;
        }
    }
}

template <int DEG, int WIN>
struct BackprojectAdamLaunch {
    static void run(dim3 grid, hipStream_t stream, float* v, const float4* cg, int64_t N,
                    const Cam& cam, const Cfg& cfg, const short4* r4, const uint32_t* ntiles,
                    float4* g4, const AdamArgs& A)
    {
        hipLaunchKernelGGL((k_backproject_adam<DEG, WIN>), grid, dim3(256), 0, stream, v, cg, N,
                           cam, cfg, r4, ntiles, g4, A);
    }
};

void launch_backproject_adam(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                             const float* cgrad, int64_t N, const Cam& cam, const Cfg& cfg,
                             const int16_t* rect, const uint32_t* ntiles, float* g2d,
                             float* const* st, const float* lr, float beta_o, float beta_s,
                             float b1, float b2, float bc1, float bc2, float eps,
                             hipStream_t stream)
{
    if (N <= 0) return;
    AdamArgs A;
    A.a = a; A.b = b; A.sh = sh; A.o = o; A.sigma = sigma;
    A.m_v = st[0]; A.s_v = st[1]; A.m_a = st[2]; A.s_a = st[3];
    A.m_b = st[4]; A.s_b = st[5]; A.m_sh = st[6]; A.s_sh = st[7];
    A.lr_v = lr[0]; A.lr_a = lr[1]; A.lr_b = lr[2]; A.lr_dc = lr[3]; A.lr_rest = lr[4];
    A.add_o = beta_o / (float)N;   // as the separate optimizer computes it
    A.beta_s = beta_s;
    A.k = AdamK{b1, b2, bc1, bc2, eps};
    const dim3 grid((unsigned)((N + 255) / 256));
    dispatch_deg_win<BackprojectAdamLaunch>(cfg.deg, cfg.window, grid, stream, v,
                                            reinterpret_cast<const float4*>(cgrad), N, cam, cfg,
                                            reinterpret_cast<const short4*>(rect), ntiles,
                                            reinterpret_cast<float4*>(g2d), A);
}

}  // namespace ts
