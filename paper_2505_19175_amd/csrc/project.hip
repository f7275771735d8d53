// project.hip -- per-triangle projection: pinhole projection, culling,
// window set-up and SH colour (forward).  One thread per triangle; geometry
// in FP64.
#include "geometry.h"
#include "ts_kernels.h"

namespace ts {

// ---------------------------------------------------------------------------
// Forward: project, cull, tight box, window coefficients, SH colour.
// ---------------------------------------------------------------------------

// Set up triangle `tri` for one camera and write entry `e` of the outputs
// (e = tri for a single view, view * N + tri in a batch).  The SH
// coefficients are loaded on first use into c (shared across views).
// WIN is the window function (TS_WINDOW_*).
template <int DEG, int WIN>
__device__ __forceinline__ void project_one(const float vv[9], float oi, float si,
                                            const float* __restrict__ sh, int64_t tri,
                                            float* c, bool& c_loaded, const Cam& cam,
                                            const Cfg& cfg, int64_t e, TriRecord* __restrict__ rec,
                                            short4* __restrict__ rect, float* __restrict__ depth,
                                            uint32_t* __restrict__ ntiles,
                                            float4* __restrict__ cgrad)
{
    Geo g;
    project_geo(vv, cam, cfg.z_near, g);
    const double zc = depth_centre(vv, cam);
    depth[e] = (float)zc;

    const double r = g.P > 0.0 ? fabs(g.S) / g.P : 0.0;
    // the sigmoid stays below 1, so it needs o > alpha_min strictly
    const bool o_ok = WIN == TS_WINDOW_SIGMOID ? oi > cfg.alpha_min : oi >= cfg.alpha_min;
    bool vis = g.front && (r >= (double)cfg.r_min) && o_ok && (si > 0.f);
    if (vis && !c_loaded) {
        // Issue the SH row loads before the costly tight-box set-up, so they are
        // in flight during it, for triangles whose full box holds a pixel
        // centre (the tight box lies inside it: only triangles culled later by
        // the tight box waste a load)
        const double x0 = fmin(fmin(g.q[0][0], g.q[1][0]), g.q[2][0]);
        const double x1 = fmax(fmax(g.q[0][0], g.q[1][0]), g.q[2][0]);
        const double y0 = fmin(fmin(g.q[0][1], g.q[1][1]), g.q[2][1]);
        const double y1 = fmax(fmax(g.q[0][1], g.q[1][1]), g.q[2][1]);
        const bool pre = fmax(0.0, ceil(x0 - 0.5)) <= fmin((double)(cam.W - 1), floor(x1 - 0.5)) &&
                         fmax(0.0, ceil(y0 - 0.5)) <= fmin((double)(cam.H - 1), floor(y1 - 0.5));
        if (pre) {
            load_sh<DEG>(sh, tri, c);
            c_loaded = true;
        }
    }

    // Tight region {o I >= alpha_min} = {u_k >= u_min for every k}: the
    // triangle scaled about its incentre by f = 1 - u_min / u(s), u(s) = 1
    // for Eq. 1 and r for the distance form.
    //   Eq. 1:    u_min = (alpha_min/o)^(1/sigma)
    //   sigmoid:  o sigmoid(d/sigma) >= alpha_min  <=>  d >= -sigma ln(o/alpha_min - 1)
    //             (negative: the region reaches past the triangle); nothing
    //             is left when that bound reaches r, everything when
    //             alpha_min = 0
    //   LSE:      phi_lse >= phi_max, so the region lies in {phi_max <=
    //             u_min phi_lse(s)}: a distance bound of u_min (r - ln 3)
    int px0 = 0, px1 = -1, py0 = 0, py1 = -1;
    double umin = 0.0, phis = 0.0;
    bool whole = false;   // unbounded support: the whole image
    if (vis) {
        const double sx = (g.len[1] * g.q[0][0] + g.len[2] * g.q[1][0] + g.len[0] * g.q[2][0]) / g.P;
        const double sy = (g.len[1] * g.q[0][1] + g.len[2] * g.q[1][1] + g.len[0] * g.q[2][1]) / g.P;
        double f;
        if constexpr (WIN == TS_WINDOW_SIGMOID) {
            if (cfg.alpha_min > 0.f) {
                umin = -(double)si * log((double)oi / (double)cfg.alpha_min - 1.0);
                vis = umin < r;
            } else {
                whole = true;
                umin = -INFINITY;
            }
            f = whole ? 1.0 : 1.0 - umin / r;
        } else if constexpr (WIN == TS_WINDOW_LSE) {
            phis = kLn3 - r;
            vis = phis < 0.0;
            umin = pow((double)cfg.alpha_min / (double)oi, 1.0 / (double)si) * (r - kLn3);
            f = 1.0 - umin / r;
        } else {
            umin = pow((double)cfg.alpha_min / (double)oi, 1.0 / (double)si);
            f = 1.0 - umin;
        }
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double x = fma(f, g.q[j][0] - sx, sx);
            const double y = fma(f, g.q[j][1] - sy, sy);
            xmin = fmin(xmin, x); xmax = fmax(xmax, x);
            ymin = fmin(ymin, y); ymax = fmax(ymax, y);
        }
        if (whole) {
            xmin = ymin = -1e300;
            xmax = ymax = 1e300;
        }
        const double fx0 = fmax(0.0, ceil(xmin - 0.5));
        const double fx1 = fmin((double)(cam.W - 1), floor(xmax - 0.5));
        const double fy0 = fmax(0.0, ceil(ymin - 0.5));
        const double fy1 = fmin((double)(cam.H - 1), floor(ymax - 0.5));
        if (vis && fx0 <= fx1 && fy0 <= fy1) {   // false for NaN as well
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
    // u_k(p) = w_k cross(e_k, p - q_k), w_k = P / (2A l_k) (Eq. 1) or
    // sgn(2A) / l_k (distance form), relative to the anchor
    const double ax = (double)px0, ay = (double)py0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double w = WIN == TS_WINDOW_PAPER ? g.P / (g.S * g.len[k])
                                                : (g.S > 0.0 ? 1.0 : -1.0) / g.len[k];
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
    // rounded toward zero so the bound stays below u_min.  The sigmoid's
    // bound can be near zero or negative: it keeps a margin of
    // (|u_min| + sigma) 2^-10 pixels, rounded down.
    if constexpr (WIN == TS_WINDOW_SIGMOID)
        R.ut = whole ? -INFINITY
                     : __double2float_rd(umin - (fabs(umin) + (double)si) * (1.0 / 1024.0));
    else
        R.ut = __double2float_rz(umin * (1.0 - 1.0 / 1024.0));
    R.phis = (float)phis;
    R.pad[0] = R.pad[1] = 0.f;

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

    if (cgrad) {
        // what the backward needs of the colour: the channels not clamped at
        // zero and J[c][b] = sum_k sh_kc dY_k/d dir_b, so it never re-reads SH
        float dY[16][3], J[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        sh_basis_grad(DEG, (float)d[0], (float)d[1], (float)d[2], dY);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
#pragma unroll
                for (int b = 0; b < 3; ++b) J[ch][b] = fmaf(c[3 * k + ch], dY[k][b], J[ch][b]);
        const uint32_t open = (acc[0] > 0.f ? 1u : 0u) | (acc[1] > 0.f ? 2u : 0u) |
                              (acc[2] > 0.f ? 4u : 0u);
        cgrad[3 * e + 0] = make_float4(J[0][0], J[0][1], J[0][2], J[1][0]);
        cgrad[3 * e + 1] = make_float4(J[1][1], J[1][2], J[2][0], J[2][1]);
        cgrad[3 * e + 2] = make_float4(J[2][2], __uint_as_float(open), 0.f, 0.f);
    }
}

template <int DEG, int WIN>
__global__ __launch_bounds__(256) void k_project(
    const float* __restrict__ v, const float* __restrict__ o, const float* __restrict__ sigma,
    const float* __restrict__ sh, int64_t N, Cam cam, Cfg cfg, TriRecord* __restrict__ rec,
    short4* __restrict__ rect, float* __restrict__ depth, uint32_t* __restrict__ ntiles,
    float4* __restrict__ cgrad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float vv[9], c[3 * (DEG + 1) * (DEG + 1)];
    bool c_loaded = false;
    load_vertices(v, i, vv);
    project_one<DEG, WIN>(vv, o[i], sigma[i], sh, i, c, c_loaded, cam, cfg, i, rec, rect, depth,
                          ntiles, cgrad);
}

// All views of a batch: each triangle is read once (vertices, opacity,
// sigma, and its SH row only if some view keeps it) and set up per view.
template <int DEG, int WIN>
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
        project_one<DEG, WIN>(vv, oi, si, sh, i, c, c_loaded, cam, cfg, (int64_t)view * N + i,
                              rec, rect, depth, ntiles, nullptr);
    }
}

template <int DEG, int WIN>
struct ProjectLaunch {
    static void run(dim3 grid, hipStream_t stream, const float* v, const float* o,
                    const float* sigma, const float* sh, int64_t N, const Cam& cam,
                    const Cfg& cfg, TriRecord* r, short4* r4, float* depth, uint32_t* ntiles,
                    float4* cg)
    {
        hipLaunchKernelGGL((k_project<DEG, WIN>), grid, dim3(256), 0, stream, v, o, sigma, sh, N,
                           cam, cfg, r, r4, depth, ntiles, cg);
    }
};

template <int DEG, int WIN>
struct ProjectViewsLaunch {
    static void run(dim3 grid, hipStream_t stream, const float* v, const float* o,
                    const float* sigma, const float* sh, int64_t N, const ts_view* views,
                    const uint32_t* ctl, const Cfg& cfg, TriRecord* r, short4* r4, float* depth,
                    uint32_t* ntiles)
    {
        hipLaunchKernelGGL((k_project_views<DEG, WIN>), grid, dim3(256), 0, stream, v, o, sigma,
                           sh, N, views, ctl, cfg, r, r4, depth, ntiles);
    }
};

void launch_project(const float* v, const float* o, const float* sigma, const float* sh,
                    int64_t N, const Cam& cam, const Cfg& cfg, void* rec, int16_t* rect,
                    float* depth, uint32_t* ntiles, float* cgrad, hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256));
    dispatch_deg_win<ProjectLaunch>(cfg.deg, cfg.window, grid, stream, v, o, sigma, sh, N, cam,
                                    cfg, reinterpret_cast<TriRecord*>(rec),
                                    reinterpret_cast<short4*>(rect), depth, ntiles,
                                    reinterpret_cast<float4*>(cgrad));
}

void launch_project_views(const float* v, const float* o, const float* sigma, const float* sh,
                          int64_t N, const ts_view* views, const uint32_t* ctl, const Cfg& cfg,
                          void* rec, int16_t* rect, float* depth, uint32_t* ntiles,
                          hipStream_t stream)
{
    const dim3 grid((unsigned)((N + 255) / 256));
    dispatch_deg_win<ProjectViewsLaunch>(cfg.deg, cfg.window, grid, stream, v, o, sigma, sh, N,
                                         views, ctl, cfg, reinterpret_cast<TriRecord*>(rec),
                                         reinterpret_cast<short4*>(rect), depth, ntiles);
}

}  // namespace ts
