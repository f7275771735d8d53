// train.hip -- the pieces of a training step around the renderer (Sec. 3.3):
// the photometric loss (1 - lambda) L1 + lambda (1 - SSIM) and its image
// gradient, the opacity and size losses, and Adam on the raw parameters.
//
// SSIM uses local statistics under an 11x11 Gaussian window; each of the two
// SSIM kernels stages a 26x26 patch (a 16x16 tile and its 5-pixel halo,
// zeros outside the image) in LDS and applies the separable window as a
// row pass and a column pass.  Both are stencils bound by LDS traffic and
// HBM; the optimizer kernels stream every parameter array once (HBM).
#include <math.h>

#include "adam.h"
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

constexpr int kS = 16;            // output tile
constexpr int kR = 5;             // window radius
constexpr int kP = kS + 2 * kR;   // staged patch width
constexpr int kPS = 28;           // row stride of a staged patch: whole 16-byte vectors
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win11 {
    float w[11];
};

// Row pass then column pass of the separable window over NQ staged
// quantities: in[q][26][26] -> out[q] at this thread's pixel (ty, tx).
// Each pass is register-blocked: one thread loads a whole staged row (or
// column) once and produces its 16 outputs, so LDS reads drop from 11 per
// output to under 2.
template <int NQ>
__device__ __forceinline__ void blur_patch(float (*in)[kP][kPS], float (*row)[kP][kS],
                                           float (*col)[kS][kS], const Win11& W, int tx, int ty,
                                           float* out)
{
    const int t = threadIdx.x;
    if (t < NQ * kP) {   // row job (q, r)
        const int q = t / kP, r = t - q * kP;
        float v[kPS];
        const float4* src = reinterpret_cast<const float4*>(&in[q][r][0]);
#pragma unroll
        for (int c4 = 0; c4 < kPS / 4; ++c4) {
            const float4 x = src[c4];
            v[4 * c4] = x.x; v[4 * c4 + 1] = x.y; v[4 * c4 + 2] = x.z; v[4 * c4 + 3] = x.w;
        }
        float4* dst = reinterpret_cast<float4*>(&row[q][r][0]);
#pragma unroll
        for (int c4 = 0; c4 < kS / 4; ++c4) {
            float o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < 11; ++k) acc = fmaf(W.w[k], v[4 * c4 + j + k], acc);
                o[j] = acc;
            }
            dst[c4] = make_float4(o[0], o[1], o[2], o[3]);
        }
    }
    __syncthreads();
    if (t < NQ * kS) {   // column job (q, c)
        const int q = t / kS, c = t - q * kS;
        float v[kP];
#pragma unroll
        for (int r = 0; r < kP; ++r) v[r] = row[q][r][c];
#pragma unroll
        for (int y = 0; y < kS; ++y) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) acc = fmaf(W.w[k], v[y + k], acc);
            col[q][y][c] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = col[q][ty][tx];
}

// Per pixel and channel: SSIM and the coefficients of its gradient,
//   d_mx = dS/dmu_x - 2 mu_x dS/dvar_x - mu_y dS/dcov,  d_exx = dS/dvar_x,
//   d_exy = dS/dcov,
// scaled by the upstream -lambda / n; and the per-workgroup sums of |x - y|
// and S (the loss value).
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x_img,
                                                  const float* __restrict__ y_img, int W, int H,
                                                  Win11 win, float up, float* __restrict__ coef,
                                                  float* __restrict__ part)
{
    __shared__ __align__(16) float in[5][kP][kPS];
    __shared__ __align__(16) float row[5][kP][kS];
    __shared__ float col[5][kS][kS];
    __shared__ float red[2][8];
    const int ch = blockIdx.z;
    const int64_t hw = (int64_t)W * H;
    const float* xc = x_img + ch * hw;
    const float* yc = y_img + ch * hw;
    const int x0 = blockIdx.x * kS - kR, y0 = blockIdx.y * kS - kR;
    for (int e = threadIdx.x; e < kP * kP; e += 256) {
        const int r = e / kP, c = e % kP, gx = x0 + c, gy = y0 + r;
        const bool ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const float a = ok ? xc[(int64_t)gy * W + gx] : 0.f;
        const float b = ok ? yc[(int64_t)gy * W + gx] : 0.f;
        in[0][r][c] = a;
        in[1][r][c] = b;
        in[2][r][c] = a * a;
        in[3][r][c] = b * b;
        in[4][r][c] = a * b;
    }
    __syncthreads();
    const int tx = threadIdx.x % kS, ty = threadIdx.x / kS;
    float m[5];
    blur_patch<5>(in, row, col, win, tx, ty, m);
    const int px = blockIdx.x * kS + tx, py = blockIdx.y * kS + ty;
    const bool inside = px < W && py < H;
    float l1 = 0.f, s = 0.f;
    if (inside) {
        const float mx = m[0], my = m[1];
        const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        const float A = 2.f * mx * my + kC1, Bn = 2.f * cxy + kC2;
        const float D1 = mx * mx + my * my + kC1, D2 = vx + vy + kC2;
        const float inv = 1.f / (D1 * D2);
        s = A * Bn * inv;
        const float dmx = 2.f * my * Bn * inv - s * 2.f * mx / D1;
        const float dvx = -s / D2;
        const float dcv = 2.f * A * inv;
        const int64_t p = (int64_t)py * W + px;
        float* cc = coef + ch * 3 * hw;
        cc[p] = up * (dmx - 2.f * mx * dvx - my * dcv);
        cc[hw + p] = up * dvx;
        cc[2 * hw + p] = up * dcv;
        l1 = fabsf(in[0][ty + kR][tx + kR] - in[1][ty + kR][tx + kR]);
    }
    // workgroup sums (wave reduction, then one value per wave)
    for (int o = 32; o > 0; o >>= 1) {
        l1 += __shfl_xor(l1, o);
        s += __shfl_xor(s, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = l1;
        red[1][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[2 * b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        part[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// loss[0] = mean |x - y|, loss[1] = mean SSIM, from the per-workgroup sums
// (one workgroup, fixed order: reproducible).  s holds 2 x 256 doubles.
__device__ void loss_total(const float* __restrict__ part, int64_t nb, double n,
                           float* __restrict__ loss, double (*s)[256])
{
    double a = 0.0, b = 0.0;
    for (int64_t j = threadIdx.x; j < nb; j += 256) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s[0][threadIdx.x] += s[0][threadIdx.x + h];
            s[1][threadIdx.x] += s[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = (float)(s[0][0] / n);
        loss[1] = (float)(s[1][0] / n);
    }
}

// dL/dC = (1 - lambda) sign(x - y) / n + blur(d_mx) + 2 x blur(d_exx) + y blur(d_exy).
// With loss set, the grid has a fourth z-plane whose first workgroup sums
// the forward's partial sums into the loss value (the other workgroups of
// that plane exit): the reduction runs beside the gradient tiles instead of
// in a launch of its own.
__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x_img,
                                                  const float* __restrict__ y_img, int W, int H,
                                                  Win11 win, float l1w,
                                                  const float* __restrict__ coef,
                                                  float* __restrict__ grad,
                                                  const float* __restrict__ part, double n,
                                                  float* __restrict__ loss)
{
    __shared__ __align__(16) float in[3][kP][kPS];
    __shared__ __align__(16) float row[3][kP][kS];
    __shared__ float col[3][kS][kS];
    static_assert(sizeof(in) >= 2 * 256 * sizeof(double), "reduction scratch");
    if (blockIdx.z == 3) {
        if (blockIdx.x == 0 && blockIdx.y == 0)
            loss_total(part, (int64_t)gridDim.x * gridDim.y * 3, n, loss,
                       reinterpret_cast<double (*)[256]>(&in[0][0][0]));
        return;
    }
    const int ch = blockIdx.z;
    const int64_t hw = (int64_t)W * H;
    const float* cc = coef + ch * 3 * hw;
    const int x0 = blockIdx.x * kS - kR, y0 = blockIdx.y * kS - kR;
    for (int e = threadIdx.x; e < kP * kP; e += 256) {
        const int r = e / kP, c = e % kP, gx = x0 + c, gy = y0 + r;
        const bool ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const int64_t p = (int64_t)gy * W + gx;
        in[0][r][c] = ok ? cc[p] : 0.f;
        in[1][r][c] = ok ? cc[hw + p] : 0.f;
        in[2][r][c] = ok ? cc[2 * hw + p] : 0.f;
    }
    __syncthreads();
    const int tx = threadIdx.x % kS, ty = threadIdx.x / kS;
    float b[3];
    blur_patch<3>(in, row, col, win, tx, ty, b);
    const int px = blockIdx.x * kS + tx, py = blockIdx.y * kS + ty;
    if (px >= W || py >= H) return;
    const int64_t p = ch * hw + (int64_t)py * W + px;
    const float x = x_img[p], y = y_img[p];
    const float sg = x > y ? 1.f : (x < y ? -1.f : 0.f);
    grad[p] = fmaf(l1w, sg, b[0] + 2.f * x * b[1] + y * b[2]);
}

size_t image_loss_workspace_bytes(int W, int H)
{
    const int64_t tiles = (int64_t)((W + kS - 1) / kS) * ((H + kS - 1) / kS) * 3;
    return (size_t)(9 * (int64_t)W * H * 4 + tiles * 8 + 256);
}

void launch_image_loss(const float* rgb, const float* target, int W, int H, float lambda,
                       float* grad, float* loss, void* ws, hipStream_t stream)
{
    Win11 win;
    double g[11], sum = 0.0;
    for (int k = 0; k < 11; ++k) {
        const double d = k - 5;
        g[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < 11; ++k) win.w[k] = (float)(g[k] / sum);
    const double n = 3.0 * W * H;
    const dim3 grid((W + kS - 1) / kS, (H + kS - 1) / kS, 3);
    float* coef = reinterpret_cast<float*>(ws);
    float* part = coef + 9 * (int64_t)W * H;
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, stream, rgb, target, W, H, win,
                       (float)(-lambda / n), coef, part);
    const dim3 grid_b(grid.x, grid.y, loss ? 4 : 3);
    hipLaunchKernelGGL(k_ssim_bwd, grid_b, dim3(256), 0, stream, rgb, target, W, H, win,
                       (float)((1.0 - lambda) / n), coef, grad, part, n, loss);
}

// ---------------------------------------------------------------------------
// Adam with the regularizers and the activation chain folded in (the
// arithmetic is in adam.h, shared with the backward projection's fused step).
// ---------------------------------------------------------------------------

// Vertices: the block's 256 vertex and gradient rows are staged through LDS
// so every global access is coalesced; each thread adds its triangle's
// size-loss gradient in LDS, then the update runs element-wise.
__global__ __launch_bounds__(256) void k_adam_vertices(float* __restrict__ v,
                                                       const float* __restrict__ gv,
                                                       float* __restrict__ m, float* __restrict__ s,
                                                       int64_t N, float beta_s, float lr, AdamK k)
{
    __shared__ float sv[256 * 9], sg[256 * 9];
    const int64_t base = (int64_t)blockIdx.x * 256;
    const int nt = (int)min((int64_t)256, N - base);
    const int n = 9 * nt;
    const int64_t off = 9 * base;
    for (int f = threadIdx.x; f < n; f += 256) {
        sv[f] = v[off + f];
        sg[f] = gv[off + f];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < nt && beta_s != 0.f) size_loss_grad(sv + 9 * t, sg + 9 * t, beta_s, N);
    __syncthreads();
    for (int f = threadIdx.x; f < n; f += 256) {
        float mi = m[off + f], si = s[off + f];
        v[off + f] = adam_update(sv[f], sg[f], mi, si, lr, k);
        m[off + f] = mi;
        s[off + f] = si;
    }
}

// Flat Adam; element e uses lr_a when e % row < first, else lr_b; act as in
// act_grad (0: g as given); with act 1 or 2, out[e] holds the activated old
// value and becomes the activated new one.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ s,
                                              int64_t n, int row, int first, float lr_a, float lr_b,
                                              AdamK k, int act, float add,
                                              float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gi = act != 0 ? act_grad(g[e], act, add, out[e]) : g[e];
    float mi = m[e], si = s[e];
    const float lr = (int)(e % row) < first ? lr_a : lr_b;
    const float pi = adam_update(p[e], gi, mi, si, lr, k);
    m[e] = mi;
    s[e] = si;
    p[e] = pi;
    if (act != 0) out[e] = act_value(pi, act);
}

void launch_optimizer(float* v, float* a, float* b, float* sh, float* o, float* sigma, int nsh,
                      int64_t N, const float* gv, const float* go, const float* gs,
                      const float* gsh, float* const* st, const float* lr, float beta_o,
                      float beta_s, float b1, float b2, float bc1, float bc2, float eps,
                      hipStream_t stream)
{
    if (N <= 0) return;
    const AdamK k{b1, b2, bc1, bc2, eps};
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_adam_vertices, dim3(nb), dim3(256), 0, stream, v, gv, st[0], st[1], N,
                       beta_s, lr[0], k);
    hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, stream, a, go, st[2], st[3], N, 1, 1,
                       lr[1], lr[1], k, 1, beta_o / (float)N, o);
    hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, stream, b, gs, st[4], st[5], N, 1, 1,
                       lr[2], lr[2], k, 2, 0.f, sigma);
    const int64_t n = (int64_t)nsh * N;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh, gsh,
                       st[6], st[7], n, nsh, 3, lr[3], lr[4], k, 0, 0.f, nullptr);
}

}  // namespace ts
