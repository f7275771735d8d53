// project.hip -- per-triangle kernels: projection + window set-up + SH colour
// (forward) and the chain from 2D gradients to the triangle parameters
// (backward).  One thread per triangle; geometry in FP64.
#include "ts_device.h"
#include "ts_kernels.h"

namespace ts {

// Camera-space and projected vertices with the edge quantities every
// consumer needs.  Edge k runs from q_k to q_{k+1}.
struct Geo {
    double xc[3][3];
    double q[3][2];
    double e[3][2];
    double len[3];
    double S;     // signed doubled area
    double P;     // perimeter
    bool front;   // every vertex beyond the near plane
};

__device__ __forceinline__ void load_vertices(const float* __restrict__ v, int64_t i, float vv[9])
{
    const float* p = v + 9 * i;
#pragma unroll
    for (int a = 0; a < 9; ++a) vv[a] = p[a];
}

__device__ __forceinline__ void project_geo(const float vv[9], const Cam& cam, float z_near, Geo& g)
{
    g.front = true;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double acc = (double)cam.t[a];
            acc = fma((double)cam.R[3 * a + 0], (double)vv[3 * j + 0], acc);
            acc = fma((double)cam.R[3 * a + 1], (double)vv[3 * j + 1], acc);
            acc = fma((double)cam.R[3 * a + 2], (double)vv[3 * j + 2], acc);
            g.xc[j][a] = acc;
        }
        g.front = g.front && (g.xc[j][2] > (double)z_near);
        const double iz = 1.0 / g.xc[j][2];
        g.q[j][0] = fma((double)cam.fx * g.xc[j][0], iz, (double)cam.cx);
        g.q[j][1] = fma((double)cam.fy * g.xc[j][1], iz, (double)cam.cy);
    }
    g.P = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        g.e[k][0] = g.q[k1][0] - g.q[k][0];
        g.e[k][1] = g.q[k1][1] - g.q[k][1];
        g.len[k] = sqrt(g.e[k][0] * g.e[k][0] + g.e[k][1] * g.e[k][1]);
        g.P += g.len[k];
    }
    // 2A = cross(q1 - q0, q2 - q0)
    g.S = g.e[0][0] * (g.q[2][1] - g.q[0][1]) - g.e[0][1] * (g.q[2][0] - g.q[0][0]);
}

// Depth key: mean camera-space z of the three vertices, every operation
// rounded in the written order (no contraction), so the float32 key is a
// fixed function of the inputs: z_j = ((R20 v0 + R21 v1) + R22 v2) + t2,
// z_c = ((z_0 + z_1) + z_2) / 3.
__device__ __forceinline__ double depth_centre(const float vv[9], const Cam& cam)
{
    double zs = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double z = __dmul_rn((double)cam.R[6], (double)vv[3 * j + 0]);
        z = __dadd_rn(z, __dmul_rn((double)cam.R[7], (double)vv[3 * j + 1]));
        z = __dadd_rn(z, __dmul_rn((double)cam.R[8], (double)vv[3 * j + 2]));
        z = __dadd_rn(z, (double)cam.t[2]);
        zs = j == 0 ? z : __dadd_rn(zs, z);
    }
    return zs / 3.0;
}

// Unit direction from the camera centre -R^T t to the centroid, and its norm.
__device__ __forceinline__ void view_dir(const float vv[9], const Cam& cam, double d[3], double& nrm)
{
    double dv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double cen = ((double)vv[a] + (double)vv[3 + a] + (double)vv[6 + a]) * (1.0 / 3.0);
        const double cc = -((double)cam.R[a] * cam.t[0] + (double)cam.R[3 + a] * cam.t[1] +
                            (double)cam.R[6 + a] * cam.t[2]);
        dv[a] = cen - cc;
    }
    nrm = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = dv[a] / nrm;
}

// ---------------------------------------------------------------------------
// Forward: project, cull, tight box, window coefficients, SH colour.
// ---------------------------------------------------------------------------
template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t i, float* c);

// Set up triangle `tri` for one camera and write entry `e` of the outputs
// (e = tri for a single view, view * N + tri in a batch).  The SH
// coefficients are loaded on first use into c (shared across views).
template <int DEG>
__device__ __forceinline__ void project_one(const float vv[9], float oi, float si,
                                            const float* __restrict__ sh, int64_t tri,
                                            float* c, bool& c_loaded, const Cam& cam,
                                            const Cfg& cfg, int64_t e, TriRecord* __restrict__ rec,
                                            short4* __restrict__ rect, float* __restrict__ depth,
                                            uint32_t* __restrict__ ntiles, float4* __restrict__ g2d)
{
    Geo g;
    project_geo(vv, cam, cfg.z_near, g);
    const double zc = depth_centre(vv, cam);
    depth[e] = (float)zc;

    const double r = g.P > 0.0 ? fabs(g.S) / g.P : 0.0;
    bool vis = g.front && (r >= (double)cfg.r_min) && (oi >= cfg.alpha_min) && (si > 0.f);

    // Tight region {o I >= alpha_min} = {u >= u_min}: the triangle scaled
    // about its incentre by 1 - u_min, u_min = (alpha_min/o)^(1/sigma).
    int px0 = 0, px1 = -1, py0 = 0, py1 = -1;
    double umin = 0.0;
    if (vis) {
        const double sx = (g.len[1] * g.q[0][0] + g.len[2] * g.q[1][0] + g.len[0] * g.q[2][0]) / g.P;
        const double sy = (g.len[1] * g.q[0][1] + g.len[2] * g.q[1][1] + g.len[0] * g.q[2][1]) / g.P;
        umin = pow((double)cfg.alpha_min / (double)oi, 1.0 / (double)si);
        const double f = 1.0 - umin;
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double x = fma(f, g.q[j][0] - sx, sx);
            const double y = fma(f, g.q[j][1] - sy, sy);
            xmin = fmin(xmin, x); xmax = fmax(xmax, x);
            ymin = fmin(ymin, y); ymax = fmax(ymax, y);
        }
        const double fx0 = fmax(0.0, ceil(xmin - 0.5));
        const double fx1 = fmin((double)(cam.W - 1), floor(xmax - 0.5));
        const double fy0 = fmax(0.0, ceil(ymin - 0.5));
        const double fy1 = fmin((double)(cam.H - 1), floor(ymax - 0.5));
        if (fx0 <= fx1 && fy0 <= fy1) {   // false for NaN as well
            px0 = (int)fx0; px1 = (int)fx1; py0 = (int)fy0; py1 = (int)fy1;
        } else {
            vis = false;
        }
    }
    if (!vis) {
        ntiles[e] = 0u;
        rect[e] = make_short4(0, -1, 0, -1);
        return;
    }
    rect[e] = make_short4((short)px0, (short)px1, (short)py0, (short)py1);
    ntiles[e] = (uint32_t)((px1 / kTile - px0 / kTile + 1) * (py1 / kTile - py0 / kTile + 1));

    TriRecord R;
    // u_k(p) = w_k cross(e_k, p - q_k), w_k = P / (2A l_k), relative to the anchor
    const double ax = (double)px0, ay = (double)py0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double w = g.P / (g.S * g.len[k]);
        const double qx = g.q[k][0] - ax, qy = g.q[k][1] - ay;
        R.A[k] = -w * g.e[k][1];
        R.B[k] = w * g.e[k][0];
        R.C[k] = w * (g.e[k][0] * (0.5 - qy) - g.e[k][1] * (0.5 - qx));
    }
    R.ax = (int16_t)px0;
    R.ay = (int16_t)py0;
    R.o = oi;
    R.sigma = si;
    R.z = (float)zc;
    R.px0 = (int16_t)px0; R.px1 = (int16_t)px1; R.py0 = (int16_t)py0; R.py1 = (int16_t)py1;
    R.tri = (uint32_t)tri;
    // A pixel with u below u_min (1 - 2^-10) cannot reach alpha_min through the
    // FP32 window (its error is orders of magnitude below that margin);
    // rounded toward zero so the bound stays below u_min.
    R.ut = __double2float_rz(umin * (1.0 - 1.0 / 1024.0));
    R.pad[0] = R.pad[1] = R.pad[2] = 0.f;

    // colour: real SH along the view direction, + 1/2, clamped at zero
    double d[3], nrm;
    view_dir(vv, cam, d, nrm);
    constexpr int K = (DEG + 1) * (DEG + 1);
    float Y[16];
    sh_basis(DEG, (float)d[0], (float)d[1], (float)d[2], Y);
    if (!c_loaded) {
        load_sh<DEG>(sh, tri, c);
        c_loaded = true;
    }
    float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[0] = fmaf(c[3 * k + 0], Y[k], acc[0]);
        acc[1] = fmaf(c[3 * k + 1], Y[k], acc[1]);
        acc[2] = fmaf(c[3 * k + 2], Y[k], acc[2]);
    }
    R.rgb[0] = fmaxf(acc[0], 0.f);
    R.rgb[1] = fmaxf(acc[1], 0.f);
    R.rgb[2] = fmaxf(acc[2], 0.f);

    const float4* src = reinterpret_cast<const float4*>(&R);
    float4* dst = reinterpret_cast<float4*>(rec + e);
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[j] = src[j];
    if (g2d) {
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 4; ++j) g2d[4 * e + j] = z4;
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(
    const float* __restrict__ v, const float* __restrict__ o, const float* __restrict__ sigma,
    const float* __restrict__ sh, int64_t N, Cam cam, Cfg cfg, TriRecord* __restrict__ rec,
    short4* __restrict__ rect, float* __restrict__ depth, uint32_t* __restrict__ ntiles,
    float4* __restrict__ g2d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float vv[9], c[3 * (DEG + 1) * (DEG + 1)];
    bool c_loaded = false;
    load_vertices(v, i, vv);
    project_one<DEG>(vv, o[i], sigma[i], sh, i, c, c_loaded, cam, cfg, i, rec, rect, depth,
                     ntiles, g2d);
}

// All views of a batch: each triangle is read once (vertices, opacity,
// sigma, and its SH row only if some view keeps it) and set up per view.
template <int DEG>
__global__ __launch_bounds__(256) void k_project_views(
    const float* __restrict__ v, const float* __restrict__ o, const float* __restrict__ sigma,
    const float* __restrict__ sh, int64_t N, const ts_view* __restrict__ views,
    const uint32_t* __restrict__ ctl, Cfg cfg, TriRecord* __restrict__ rec,
    short4* __restrict__ rect, float* __restrict__ depth, uint32_t* __restrict__ ntiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t nviews = ctl[0];
    float vv[9], c[3 * (DEG + 1) * (DEG + 1)];
    bool c_loaded = false;
    load_vertices(v, i, vv);
    const float oi = o[i], si = sigma[i];
    for (uint32_t view = 0; view < nviews; ++view) {
        const ts_camera& vc = views[view].cam;
        Cam cam;
#pragma unroll
        for (int a = 0; a < 9; ++a) cam.R[a] = vc.R[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) cam.t[a] = vc.t[a];
        cam.fx = vc.fx; cam.fy = vc.fy; cam.cx = vc.cx; cam.cy = vc.cy;
        cam.W = vc.width; cam.H = vc.height;
        project_one<DEG>(vv, oi, si, sh, i, c, c_loaded, cam, cfg, (int64_t)view * N + i, rec,
                         rect, depth, ntiles, nullptr);
    }
}

// Coefficients of one triangle: float4 loads when the row is 16-byte aligned.
template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t i, float* c)
{
    constexpr int NSH = 3 * (DEG + 1) * (DEG + 1);
    const float* p = sh + (int64_t)NSH * i;
    if constexpr (NSH % 4 == 0) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int j = 0; j < NSH / 4; ++j) {
            const float4 t = q[j];
            c[4 * j + 0] = t.x; c[4 * j + 1] = t.y; c[4 * j + 2] = t.z; c[4 * j + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NSH; ++j) c[j] = p[j];
    }
}

// Stores n floats of LDS to contiguous global memory, one 16-byte vector per
// lane where the block is full (n % 4 == 0 and 16-byte aligned).
__device__ __forceinline__ void block_store(float* __restrict__ dst, const float* src, int n)
{
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
        float4* d4 = reinterpret_cast<float4*>(dst);
        for (int f = threadIdx.x; f < n / 4; f += blockDim.x)
            d4[f] = make_float4(src[4 * f], src[4 * f + 1], src[4 * f + 2], src[4 * f + 3]);
    } else {
        for (int f = threadIdx.x; f < n; f += blockDim.x) dst[f] = src[f];
    }
}

// ---------------------------------------------------------------------------
// Backward: 2D accumulators -> window coefficients -> projected vertices ->
// camera space -> world vertices; colour -> SH coefficients and view
// direction.  Consumes g2d (re-zeroes it).
// g2d slots: 0-2 dL/dA_k, 3-5 dL/dB_k, 6-8 dL/dC_k, 9 dL/do, 10 dL/dsigma,
//            11-13 dL/drgb, 14 dL/dz.
// A block handles 256 consecutive triangles and writes their gradient rows
// through LDS, so every store of the block is contiguous (the SH gradient is
// the largest array the step writes: 12 (deg+1)^2 bytes per triangle).
// ---------------------------------------------------------------------------
template <int DEG>
__global__ __launch_bounds__(256) void k_backproject(
    const float* __restrict__ v, const float* __restrict__ sh, int64_t N, Cam cam, Cfg cfg,
    const short4* __restrict__ rect, const uint32_t* __restrict__ ntiles,
    float4* __restrict__ g2d, float* __restrict__ gv, float* __restrict__ go,
    float* __restrict__ gsig, float* __restrict__ gsh)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int NSH = 3 * K;
    __shared__ float s_gv[256 * 9];
    __shared__ float s_y[256 * K];     // SH basis at the view direction
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

        float vv[9];
        load_vertices(v, i, vv);
        Geo g;
        project_geo(vv, cam, cfg.z_near, g);
        const short4 rc = rect[i];
        const double ax = (double)rc.x, ay = (double)rc.z;

        // coefficients -> (w_k, e_k, q_k)
        double gq[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        double ge[3][2];
        double gP = 0.0, gS = 0.0, gl[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double w = g.P / (g.S * g.len[k]);
            const double qx = g.q[k][0] - ax, qy = g.q[k][1] - ay;
            const double ex = g.e[k][0], ey = g.e[k][1];
            const double gA = G[k], gB = G[3 + k], gC = G[6 + k];
            const double ck = ex * (0.5 - qy) - ey * (0.5 - qx);
            const double gw = -gA * ey + gB * ex + gC * ck;
            ge[k][0] = gB * w + gC * w * (0.5 - qy);
            ge[k][1] = -gA * w - gC * w * (0.5 - qx);
            gq[k][0] += gC * w * ey;
            gq[k][1] += -gC * w * ex;
            // w = P / (S l_k)
            gP += gw / (g.S * g.len[k]);
            gS += -gw * w / g.S;
            gl[k] = -gw * w / g.len[k];
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

        // colour: rgb = max(0, sum_k sh_k Y_k(d) + 1/2)
        double d[3], nrm;
        view_dir(vv, cam, d, nrm);
        const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
        float Y[16], dY[16][3], c[NSH];
        sh_basis(DEG, dx, dy, dz, Y);
        sh_basis_grad(DEG, dx, dy, dz, dY);
        load_sh<DEG>(sh, i, c);
        float raw[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            raw[0] = fmaf(c[3 * k + 0], Y[k], raw[0]);
            raw[1] = fmaf(c[3 * k + 1], Y[k], raw[1]);
            raw[2] = fmaf(c[3 * k + 2], Y[k], raw[2]);
        }
        const float gr0 = raw[0] > 0.f ? G[11] : 0.f;
        const float gr1 = raw[1] > 0.f ? G[12] : 0.f;
        const float gr2 = raw[2] > 0.f ? G[13] : 0.f;
        float gd[3] = {0.f, 0.f, 0.f};
        go3[0] = gr0; go3[1] = gr1; go3[2] = gr2;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            yo[k] = Y[k];
            const float s = gr0 * c[3 * k + 0] + gr1 * c[3 * k + 1] + gr2 * c[3 * k + 2];
            gd[0] = fmaf(s, dY[k][0], gd[0]);
            gd[1] = fmaf(s, dY[k][1], gd[1]);
            gd[2] = fmaf(s, dY[k][2], gd[2]);
        }
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
    if (i < N) {
        go[i] = go_;
        gsig[i] = gs_;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) s_gv[tid * 9 + a] = gvo[a];
#pragma unroll
    for (int a = 0; a < K; ++a) s_y[tid * K + a] = yo[a];
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
                    x[cq] = s_y[t * K + k] * s_g[t * 3 + ch];
                }
                d4[f] = make_float4(x[0], x[1], x[2], x[3]);
            }
            return;
        }
    }
    for (int f = tid; f < n; f += 256) {
        const int t = f / NSH, q = f - t * NSH, k = q / 3, ch = q - 3 * k;
        dst[f] = s_y[t * K + k] * s_g[t * 3 + ch];
    }
}

void launch_project(const float* v, const float* o, const float* sigma, const float* sh,
                    int64_t N, const Cam& cam, const Cfg& cfg, void* rec, int16_t* rect,
                    float* depth, uint32_t* ntiles, float* g2d, hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    TriRecord* r = reinterpret_cast<TriRecord*>(rec);
    short4* r4 = reinterpret_cast<short4*>(rect);
    float4* g4 = reinterpret_cast<float4*>(g2d);
    switch (cfg.deg) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, block, 0, stream, v, o, sigma, sh, N, cam, cfg, r, r4, depth, ntiles, g4); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, block, 0, stream, v, o, sigma, sh, N, cam, cfg, r, r4, depth, ntiles, g4); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, stream, v, o, sigma, sh, N, cam, cfg, r, r4, depth, ntiles, g4); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, block, 0, stream, v, o, sigma, sh, N, cam, cfg, r, r4, depth, ntiles, g4); break;
    }
}

void launch_project_views(const float* v, const float* o, const float* sigma, const float* sh,
                          int64_t N, const ts_view* views, const uint32_t* ctl, const Cfg& cfg,
                          void* rec, int16_t* rect, float* depth, uint32_t* ntiles,
                          hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    TriRecord* r = reinterpret_cast<TriRecord*>(rec);
    short4* r4 = reinterpret_cast<short4*>(rect);
    switch (cfg.deg) {
    case 0: hipLaunchKernelGGL(k_project_views<0>, grid, block, 0, stream, v, o, sigma, sh, N, views, ctl, cfg, r, r4, depth, ntiles); break;
    case 1: hipLaunchKernelGGL(k_project_views<1>, grid, block, 0, stream, v, o, sigma, sh, N, views, ctl, cfg, r, r4, depth, ntiles); break;
    case 2: hipLaunchKernelGGL(k_project_views<2>, grid, block, 0, stream, v, o, sigma, sh, N, views, ctl, cfg, r, r4, depth, ntiles); break;
    default: hipLaunchKernelGGL(k_project_views<3>, grid, block, 0, stream, v, o, sigma, sh, N, views, ctl, cfg, r, r4, depth, ntiles); break;
    }
}

void launch_backproject(const float* v, const float* sh, int64_t N, const Cam& cam,
                        const Cfg& cfg, const int16_t* rect, const uint32_t* ntiles, float* g2d,
                        float* gv, float* go, float* gsig, float* gsh, hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    const short4* r4 = reinterpret_cast<const short4*>(rect);
    float4* g4 = reinterpret_cast<float4*>(g2d);
    switch (cfg.deg) {
    case 0: hipLaunchKernelGGL(k_backproject<0>, grid, block, 0, stream, v, sh, N, cam, cfg, r4, ntiles, g4, gv, go, gsig, gsh); break;
    case 1: hipLaunchKernelGGL(k_backproject<1>, grid, block, 0, stream, v, sh, N, cam, cfg, r4, ntiles, g4, gv, go, gsig, gsh); break;
    case 2: hipLaunchKernelGGL(k_backproject<2>, grid, block, 0, stream, v, sh, N, cam, cfg, r4, ntiles, g4, gv, go, gsig, gsh); break;
    default: hipLaunchKernelGGL(k_backproject<3>, grid, block, 0, stream, v, sh, N, cam, cfg, r4, ntiles, g4, gv, go, gsig, gsh); break;
    }
}

}  // namespace ts
