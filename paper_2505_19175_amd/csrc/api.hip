// api.hip -- extern "C" entry points of libts.so: argument checks, workspace
// carve-up and kernel launches.  No allocation happens here.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "ts_device.h"
#include "ts_kernels.h"

namespace {

thread_local char g_msg[256] = "";

int fail(int code, const char* what)
{
    snprintf(g_msg, sizeof g_msg, "%s", what);
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    snprintf(g_msg, sizeof g_msg, "%s: %s", where, hipGetErrorString(e));
    return TS_EHIP;
}

bool cam_ok(const ts_camera* c)
{
    return c && c->width > 0 && c->height > 0 && c->width <= TS_MAX_IMAGE_DIM &&
           c->height <= TS_MAX_IMAGE_DIM;
}

bool cfg_ok(const ts_config* g)
{
    return g && g->sh_degree >= 0 && g->sh_degree <= TS_MAX_SH_DEGREE && g->alpha_max > 0.f &&
           g->alpha_max <= 1.f && g->alpha_min >= 0.f && g->alpha_min < g->alpha_max &&
           g->T_min >= 0.f && g->window >= TS_WINDOW_PAPER && g->window <= TS_WINDOW_LSE;
}

ts::Cam to_cam(const ts_camera* c)
{
    ts::Cam k;
    memcpy(k.R, c->R, sizeof k.R);
    memcpy(k.t, c->t, sizeof k.t);
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy;
    k.W = c->width; k.H = c->height;
    return k;
}

ts::Cfg to_cfg(const ts_config* g)
{
    ts::Cfg k;
    k.alpha_min = g->alpha_min; k.alpha_max = g->alpha_max; k.T_min = g->T_min;
    k.z_near = g->z_near; k.r_min = g->r_min; k.deg = g->sh_degree;
    k.bg[0] = g->bg[0]; k.bg[1] = g->bg[1]; k.bg[2] = g->bg[2];
    k.window = g->window;
    return k;
}

int tiles_x_of(const ts_camera* c) { return (c->width + TS_TILE - 1) / TS_TILE; }

bool proj_ok(const ts_proj* p)
{
    return p && p->rec && p->rect && p->depth && p->ntiles && p->g2d &&
           (reinterpret_cast<uintptr_t>(p->rec) & 15u) == 0 &&
           (reinterpret_cast<uintptr_t>(p->rect) & 7u) == 0 &&
           (reinterpret_cast<uintptr_t>(p->g2d) & 15u) == 0 &&
           (reinterpret_cast<uintptr_t>(p->cgrad) & 15u) == 0;
}

bool bins_ok(const ts_bins* b)
{
    return b && b->vals && b->ranges && b->d_count && b->capacity <= 0xffffffffull;
}

}  // namespace

// Scratch memory of ts_bin_sort_noalloc: a fixed device array in the code
// object, one copy per GPU, held until the process ends.  In host code its
// name is only a stand-in: kernels get the device address resolved below.
static __device__ __align__(256) unsigned char scratch[TS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per
// device (hipGetSymbolAddress with that device current) and kept.
int scratch_on_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "ts_bin_sort_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TS_EINVAL, "ts_bin_sort_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "ts_bin_sort_noalloc: hipGetSymbolAddress");
        if (!p) return fail(TS_EHIP, "ts_bin_sort_noalloc: null scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TS_OK;
}

// The per-triangle 2D gradient accumulators (ts_proj.g2d) must hold zeros
// when a raster backward starts; every backward projection consumes them and
// leaves them zero.  This host-side record of the accumulator arrays a raster
// backward has filled and no backward projection has consumed yet turns a
// second raster backward on them into TS_EINVAL instead of a silently summed
// gradient.
std::mutex g_g2d_mu;
const void* g_g2d_pending[64] = {};

bool g2d_pending(const void* g)
{
    std::lock_guard<std::mutex> lock(g_g2d_mu);
    for (const void* q : g_g2d_pending)
        if (q == g) return true;
    return false;
}

void g2d_mark(const void* g, bool pending)
{
    std::lock_guard<std::mutex> lock(g_g2d_mu);
    for (const void*& q : g_g2d_pending) {
        if (pending && q == nullptr) {
            q = g;
            return;
        }
        if (!pending && q == g) q = nullptr;
    }
}

int bin_sort(const char* name, const ts_proj* proj, int64_t N, const ts_camera* cam, void* ws,
             size_t ws_bytes, const ts_bins* out, uint32_t* h_count, hipStream_t stream)
{
    char msg[192];
    if (N < 0 || N > 0xffffffffll) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: N out of range", name), msg));
    if (!cam_ok(cam)) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad camera", name), msg));
    if (!bins_ok(out)) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad bins", name), msg));
    if (N > 0 && !proj_ok(proj)) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad projection", name), msg));
    const int num_tiles = ts_num_tiles(cam->width, cam->height);
    const ts::BinWorkspace need = ts::carve_bin_workspace(nullptr, N, out->capacity, num_tiles);
    if (!ws || ws_bytes < need.bytes)
        return fail(TS_EWORKSPACE,
                    (snprintf(msg, sizeof msg, "%s: workspace of %zu bytes needed, %zu available",
                              name, need.bytes, ws ? ws_bytes : (size_t)0), msg));
    const ts::BinWorkspace w = ts::carve_bin_workspace(ws, N, out->capacity, num_tiles);
    bool overflow = false;
    hipError_t e;
    if (N == 0) {
        // empty scene: zero counts and ranges, and a valid tile order
        ts::launch_fill_u32(out->d_count, 4, 0u, stream);
        ts::launch_fill_u32(out->ranges, 2 * (int64_t)num_tiles, 0u, stream);
        ts::launch_tile_order(out->ranges, num_tiles, nullptr, out->order, stream);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, name);
        if (h_count) {
            h_count[0] = 0;
            h_count[1] = 0;
        }
        return TS_OK;
    }
    e = ts::run_bin_sort(proj->ntiles, proj->depth, proj->rect, N, nullptr, nullptr, 0,
                         tiles_x_of(cam), num_tiles, w, *out, h_count, &overflow, stream);
    if (e != hipSuccess) return hip_fail(e, name);
    if (overflow) return fail(TS_ECAPACITY, (snprintf(msg, sizeof msg, "%s: instances exceed capacity", name), msg));
    return TS_OK;
}

}  // namespace

extern "C" {

size_t ts_proj_record_bytes(void) { return sizeof(ts::TriRecord); }

int32_t ts_num_tiles(int32_t width, int32_t height)
{
    if (width <= 0 || height <= 0) return 0;
    return ((width + TS_TILE - 1) / TS_TILE) * ((height + TS_TILE - 1) / TS_TILE);
}

size_t ts_bin_sort_workspace_bytes(int64_t N, uint64_t capacity, int32_t num_tiles)
{
    if (N < 0 || num_tiles < 0) return 0;
    return ts::carve_bin_workspace(nullptr, N, capacity, num_tiles).bytes;
}

int ts_project(const float* v, const float* o, const float* sigma, const float* sh, int64_t N,
               const ts_camera* cam, const ts_config* cfg, const ts_proj* out,
               hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || N > 0xffffffffll) return fail(TS_EINVAL, "ts_project: N out of range");
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_project: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_project: bad config");
    if (N == 0) return TS_OK;
    if (!v || !o || !sigma || !sh || !proj_ok(out))
        return fail(TS_EINVAL, "ts_project: null or misaligned pointer");
    ts::launch_project(v, o, sigma, sh, N, to_cam(cam), to_cfg(cfg), out->rec, out->rect,
                       out->depth, out->ntiles, out->cgrad, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_project");
}

int ts_bin_sort(const ts_proj* proj, int64_t N, const ts_camera* cam, void* ws, size_t ws_bytes,
                const ts_bins* out, uint32_t* h_count, hipStream_t stream)
{
    g_msg[0] = 0;
    return bin_sort("ts_bin_sort", proj, N, cam, ws, ws_bytes, out, h_count, stream);
}

int ts_bin_sort_noalloc(const ts_proj* proj, int64_t N, const ts_camera* cam, const ts_bins* out,
                        uint32_t* h_count, hipStream_t stream)
{
    g_msg[0] = 0;
    if (out && cam && N >= 0 && cam->width > 0 && cam->height > 0) {
        const size_t need =
            ts::carve_bin_workspace(nullptr, N, out->capacity, ts_num_tiles(cam->width, cam->height))
                .bytes;
        if (need > (size_t)TS_NOALLOC_SCRATCH_BYTES) {
            char msg[192];
            snprintf(msg, sizeof msg,
                     "ts_bin_sort_noalloc: %zu bytes of workspace needed for N = %lld, capacity = "
                     "%llu; the fixed scratch holds %zu",
                     need, (long long)N, (unsigned long long)out->capacity,
                     (size_t)TS_NOALLOC_SCRATCH_BYTES);
            return fail(TS_EWORKSPACE, msg);
        }
    }
    void* base = nullptr;
    const int rc = scratch_on_current_device(&base);
    if (rc != TS_OK) return rc;
    return bin_sort("ts_bin_sort_noalloc", proj, N, cam, base, (size_t)TS_NOALLOC_SCRATCH_BYTES, out,
                    h_count, stream);
}

}  // extern "C"

static int render_forward(const char* name, const ts_proj* proj, const ts_bins* bins,
                          const ts_camera* cam, const ts_config* cfg, float* rgb, float* alpha,
                          float* depth, float* T_final, uint32_t* last,
                          const ts_prune_stats* stats, hipStream_t stream)
{
    g_msg[0] = 0;
    char msg[160];
    if (!cam_ok(cam)) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad camera", name), msg));
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad config", name), msg));
    if (!bins_ok(bins) || !proj || !proj->rec)
        return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: bad projection or bins", name), msg));
    if (!rgb || !alpha || !depth || !T_final || !last)
        return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: null output", name), msg));
    if (stats && (!stats->max_weight || !stats->pixels))
        return fail(TS_EINVAL, (snprintf(msg, sizeof msg, "%s: null statistics", name), msg));
    ts::launch_raster_forward(proj->rec, bins->vals, bins->ranges, bins->order, to_cam(cam),
                              to_cfg(cfg), tiles_x_of(cam), ts_num_tiles(cam->width, cam->height),
                              rgb, alpha, depth, T_final, last, bins->blocks,
                              stats ? stats->max_weight : nullptr,
                              stats ? stats->pixels : nullptr, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, name);
}

extern "C" {

int ts_render_forward(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                      const ts_config* cfg, float* rgb, float* alpha, float* depth,
                      float* T_final, uint32_t* last, hipStream_t stream)
{
    return render_forward("ts_render_forward", proj, bins, cam, cfg, rgb, alpha, depth, T_final,
                          last, nullptr, stream);
}

int ts_render_forward_stats(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, const ts_prune_stats* stats,
                            hipStream_t stream)
{
    if (!stats) return fail(TS_EINVAL, "ts_render_forward_stats: null statistics");
    return render_forward("ts_render_forward_stats", proj, bins, cam, cfg, rgb, alpha, depth,
                          T_final, last, stats, stream);
}

int ts_prune_count_views(uint32_t* pixels, uint32_t* views, int64_t N, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || (N > 0 && (!pixels || !views)))
        return fail(TS_EINVAL, "ts_prune_count_views: bad arguments");
    ts::launch_prune_views(pixels, views, N, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_prune_count_views");
}

int ts_render_backward(const float* v, const float* o, const float* sigma, const float* sh,
                       int64_t N, const ts_proj* proj, const ts_bins* bins,
                       const ts_camera* cam, const ts_config* cfg, const float* dL_drgb,
                       const float* dL_dalpha, const float* dL_ddepth, const float* T_final,
                       const uint32_t* last, float* gv, float* go, float* gsigma, float* gsh,
                       hipStream_t stream)
{
    g_msg[0] = 0;
    (void)o;
    (void)sigma;
    if (N < 0 || N > 0xffffffffll) return fail(TS_EINVAL, "ts_render_backward: N out of range");
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_render_backward: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_render_backward: bad config");
    if (!bins_ok(bins)) return fail(TS_EINVAL, "ts_render_backward: bad bins");
    if (N > 0 && (!proj_ok(proj) || !proj->cgrad || !v || !sh || !gv || !go || !gsigma || !gsh))
        return fail(TS_EINVAL, "ts_render_backward: null pointer");
    if (!dL_drgb || !T_final || !last) return fail(TS_EINVAL, "ts_render_backward: null upstream");
    if (N == 0) return TS_OK;
    if (g2d_pending(proj->g2d))
        return fail(TS_EINVAL, "ts_render_backward: the 2D gradient accumulators still hold a "
                               "raster backward (call ts_project_backward first)");
    const ts::Cam k = to_cam(cam);
    const ts::Cfg g = to_cfg(cfg);
    ts::launch_raster_backward(proj->rec, bins->vals, bins->ranges, bins->order, k, g,
                               tiles_x_of(cam), ts_num_tiles(cam->width, cam->height), dL_drgb,
                               dL_dalpha, dL_ddepth, T_final, last, bins->blocks, proj->g2d,
                               stream);
    ts::launch_backproject(v, proj->cgrad, N, k, g, proj->rect, proj->ntiles, proj->g2d, gv, go,
                           gsigma, gsh, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_render_backward");
}

int ts_raster_backward(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                       const ts_config* cfg, const float* dL_drgb, const float* dL_dalpha,
                       const float* dL_ddepth, const float* T_final, const uint32_t* last,
                       hipStream_t stream)
{
    g_msg[0] = 0;
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_raster_backward: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_raster_backward: bad config");
    if (!bins_ok(bins) || !proj_ok(proj)) return fail(TS_EINVAL, "ts_raster_backward: bad state");
    if (!dL_drgb || !T_final || !last) return fail(TS_EINVAL, "ts_raster_backward: null upstream");
    if (g2d_pending(proj->g2d))
        return fail(TS_EINVAL, "ts_raster_backward: the 2D gradient accumulators still hold the "
                               "previous raster backward (call ts_project_backward first)");
    ts::launch_raster_backward(proj->rec, bins->vals, bins->ranges, bins->order, to_cam(cam),
                               to_cfg(cfg), tiles_x_of(cam), ts_num_tiles(cam->width, cam->height),
                               dL_drgb, dL_dalpha, dL_ddepth, T_final, last, bins->blocks,
                               proj->g2d, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ts_raster_backward");
    g2d_mark(proj->g2d, true);
    return TS_OK;
}

int ts_project_backward(const float* v, const float* sh, int64_t N, const ts_proj* proj,
                        const ts_camera* cam, const ts_config* cfg, float* gv, float* go,
                        float* gsigma, float* gsh, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || N > 0xffffffffll) return fail(TS_EINVAL, "ts_project_backward: N out of range");
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_project_backward: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_project_backward: bad config");
    if (N == 0) {
        if (proj) g2d_mark(proj->g2d, false);
        return TS_OK;
    }
    if (!proj_ok(proj) || !proj->cgrad || !v || !sh || !gv || !go || !gsigma || !gsh)
        return fail(TS_EINVAL, "ts_project_backward: null pointer");
    ts::launch_backproject(v, proj->cgrad, N, to_cam(cam), to_cfg(cfg), proj->rect, proj->ntiles,
                           proj->g2d, gv, go, gsigma, gsh, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ts_project_backward");
    g2d_mark(proj->g2d, false);
    return TS_OK;
}

size_t ts_fragment_workspace_bytes(int32_t width, int32_t height)
{
    if (width <= 0 || height <= 0) return 0;
    return ts::fragment_scan_workspace_bytes((int64_t)width * height);
}

int ts_render_forward_count(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, uint32_t* frag_count,
                            uint32_t* frag_offset, uint32_t* d_total, void* ws, size_t ws_bytes,
                            hipStream_t stream)
{
    g_msg[0] = 0;
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_render_forward_count: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_render_forward_count: bad config");
    if (!bins_ok(bins) || !proj || !proj->rec)
        return fail(TS_EINVAL, "ts_render_forward_count: bad projection or bins");
    if (!rgb || !alpha || !depth || !T_final || !last || !frag_count || !frag_offset || !d_total)
        return fail(TS_EINVAL, "ts_render_forward_count: null output");
    const int64_t npix = (int64_t)cam->width * cam->height;
    if (!ws || ws_bytes < ts::fragment_scan_workspace_bytes(npix))
        return fail(TS_EWORKSPACE, "ts_render_forward_count: workspace too small");
    ts::FragStore fs{frag_count, nullptr, nullptr, nullptr, nullptr};
    ts::launch_raster_forward_fragments(proj->rec, bins->vals, bins->ranges, bins->order,
                                        to_cam(cam), to_cfg(cfg), tiles_x_of(cam),
                                        ts_num_tiles(cam->width, cam->height), rgb, alpha, depth,
                                        T_final, last, bins->blocks, 1, fs, stream);
    ts::launch_fragment_offsets(frag_count, npix, frag_offset, d_total, ws, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_render_forward_count");
}

int ts_render_forward_store(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, const uint32_t* frag_offset,
                            uint32_t* frag_entry, float* frag_alpha, float* frag_T,
                            hipStream_t stream)
{
    g_msg[0] = 0;
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_render_forward_store: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_render_forward_store: bad config");
    if (!bins_ok(bins) || !proj || !proj->rec)
        return fail(TS_EINVAL, "ts_render_forward_store: bad projection or bins");
    if (!rgb || !alpha || !depth || !T_final || !last || !frag_offset || !frag_entry ||
        !frag_alpha || !frag_T)
        return fail(TS_EINVAL, "ts_render_forward_store: null output");
    ts::FragStore fs{nullptr, frag_offset, frag_entry, frag_alpha, frag_T};
    ts::launch_raster_forward_fragments(proj->rec, bins->vals, bins->ranges, bins->order,
                                        to_cam(cam), to_cfg(cfg), tiles_x_of(cam),
                                        ts_num_tiles(cam->width, cam->height), rgb, alpha, depth,
                                        T_final, last, bins->blocks, 2, fs, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_render_forward_store");
}

int ts_raster_backward_stored(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                              const ts_config* cfg, const float* dL_drgb, const float* dL_dalpha,
                              const float* dL_ddepth, const float* T_final, const uint32_t* last,
                              const uint32_t* frag_count, const uint32_t* frag_offset,
                              const uint32_t* frag_entry, const float* frag_alpha,
                              const float* frag_T, hipStream_t stream)
{
    g_msg[0] = 0;
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_raster_backward_stored: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_raster_backward_stored: bad config");
    if (!bins_ok(bins) || !proj_ok(proj))
        return fail(TS_EINVAL, "ts_raster_backward_stored: bad state");
    if (!dL_drgb || !T_final || !last || !frag_count || !frag_offset || !frag_entry ||
        !frag_alpha || !frag_T)
        return fail(TS_EINVAL, "ts_raster_backward_stored: null input");
    ts::FragStore fs{const_cast<uint32_t*>(frag_count), frag_offset,
                     const_cast<uint32_t*>(frag_entry), const_cast<float*>(frag_alpha),
                     const_cast<float*>(frag_T)};
    if (g2d_pending(proj->g2d))
        return fail(TS_EINVAL, "ts_raster_backward_stored: the 2D gradient accumulators still "
                               "hold the previous raster backward (call ts_project_backward first)");
    ts::launch_raster_backward(proj->rec, bins->vals, bins->ranges, bins->order, to_cam(cam),
                               to_cfg(cfg), tiles_x_of(cam), ts_num_tiles(cam->width, cam->height),
                               dL_drgb, dL_dalpha, dL_ddepth, T_final, last, bins->blocks,
                               proj->g2d, stream, &fs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ts_raster_backward_stored");
    g2d_mark(proj->g2d, true);
    return TS_OK;
}

int ts_batch_layout(ts_view* views, int32_t n, uint32_t* total_tiles, uint64_t* total_pixels)
{
    g_msg[0] = 0;
    if (!views || n < 0 || !total_tiles || !total_pixels)
        return fail(TS_EINVAL, "ts_batch_layout: bad arguments");
    uint64_t tiles = 0, pixels = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!cam_ok(&views[i].cam)) return fail(TS_EINVAL, "ts_batch_layout: bad camera");
        views[i].tile_offset = (uint32_t)tiles;
        views[i].tiles_x = (uint32_t)tiles_x_of(&views[i].cam);
        views[i].pixel_offset = pixels;
        tiles += (uint64_t)ts_num_tiles(views[i].cam.width, views[i].cam.height);
        pixels += (uint64_t)views[i].cam.width * (uint64_t)views[i].cam.height;
    }
    if (tiles > 0xffffffffull) return fail(TS_EINVAL, "ts_batch_layout: too many tiles");
    *total_tiles = (uint32_t)tiles;
    *total_pixels = pixels;
    return TS_OK;
}

size_t ts_batch_workspace_bytes(int64_t N, int32_t max_views, uint64_t capacity,
                                uint32_t max_tiles)
{
    if (N < 0 || max_views <= 0) return 0;
    return ts::carve_bin_workspace(nullptr, N * max_views, capacity, max_tiles).bytes + 256;
}

int ts_render_forward_batched(const float* v, const float* o, const float* sigma,
                              const float* sh, int64_t N, const ts_view* views,
                              const uint32_t* ctl, int32_t max_views, uint32_t max_tiles,
                              const ts_config* cfg, const ts_proj* proj, const ts_bins* bins,
                              void* ws, size_t ws_bytes, float* rgb, float* alpha, float* depth,
                              hipStream_t stream)
{
    g_msg[0] = 0;
    if (N <= 0 || max_views <= 0 || N * (int64_t)max_views > 0xffffffffll || max_tiles == 0)
        return fail(TS_EINVAL, "ts_render_forward_batched: sizes out of range");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_render_forward_batched: bad config");
    if (!v || !o || !sigma || !sh || !views || !ctl || !rgb || !alpha || !depth)
        return fail(TS_EINVAL, "ts_render_forward_batched: null pointer");
    if (!proj || !proj->rec || !proj->rect || !proj->depth || !proj->ntiles || !bins_ok(bins))
        return fail(TS_EINVAL, "ts_render_forward_batched: bad projection or bins");
    const int64_t entries = N * (int64_t)max_views;
    const ts::BinWorkspace need =
        ts::carve_bin_workspace(nullptr, entries, bins->capacity, (int64_t)max_tiles);
    if (!ws || ws_bytes < need.bytes + 256)
        return fail(TS_EWORKSPACE, "ts_render_forward_batched: workspace too small");
    const ts::BinWorkspace w = ts::carve_bin_workspace(ws, entries, bins->capacity, (int64_t)max_tiles);
    uint32_t* extra = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + need.bytes);
    uint32_t* queue = extra;        // tile queue head
    uint32_t* bctl = extra + 4;     // clamped descriptor: views, tiles, views * N
    uint32_t* n_entries = bctl + 2;
    const ts::Cfg g = to_cfg(cfg);

    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    const int workgroups = (int)std::min<int64_t>((int64_t)max_tiles, (int64_t)cus * 4);

    ts::launch_fill_u32(queue, 1, 0u, stream);
    ts::launch_batch_ctl(ctl, (uint32_t)max_views, max_tiles, N, bctl, stream);
    ts::launch_project_views(v, o, sigma, sh, N, views, bctl, g, proj->rec, proj->rect,
                             proj->depth, proj->ntiles, stream);
    bool overflow = false;
    hipError_t e = ts::run_bin_sort(proj->ntiles, proj->depth, proj->rect, entries, n_entries,
                                    views, N, 0, (int)max_tiles, w, *bins, nullptr, &overflow,
                                    stream, bctl + 1);
    if (e != hipSuccess) return hip_fail(e, "ts_render_forward_batched");
    ts::launch_raster_forward_queue(proj->rec, bins->vals, bins->ranges, bins->order, views, bctl,
                                    g, queue,
                                    workgroups, rgb, alpha, depth, stream);
    e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_render_forward_batched");
}

const char* ts_error_string(int code)
{
    switch (code) {
    case TS_OK: return "ok";
    case TS_EINVAL: return "invalid argument";
    case TS_ECAPACITY: return "instance count exceeds capacity";
    case TS_EWORKSPACE: return "workspace too small";
    case TS_EHIP: return "HIP error";
    default: return "unknown error";
    }
}

const char* ts_last_error(void) { return g_msg; }

size_t ts_image_loss_workspace_bytes(int width, int height)
{
    return width > 0 && height > 0 ? ts::image_loss_workspace_bytes(width, height) : 0;
}

int ts_image_loss(const float* rgb, const float* target, int width, int height, float lambda,
                  float* dL_drgb, float* loss, void* ws, size_t ws_bytes, hipStream_t stream)
{
    g_msg[0] = 0;
    if (width <= 0 || height <= 0 || width > TS_MAX_IMAGE_DIM || height > TS_MAX_IMAGE_DIM ||
        !(lambda >= 0.f && lambda <= 1.f))
        return fail(TS_EINVAL, "ts_image_loss: bad size or lambda");
    if (!rgb || !target || !dL_drgb || !ws) return fail(TS_EINVAL, "ts_image_loss: null pointer");
    if (ws_bytes < ts::image_loss_workspace_bytes(width, height))
        return fail(TS_EWORKSPACE, "ts_image_loss: workspace too small");
    ts::launch_image_loss(rgb, target, width, height, lambda, dL_drgb, loss, ws, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_image_loss");
}

int ts_optimizer_step(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                      int sh_degree, int64_t N, float* gv, float* go, float* gsigma, float* gsh,
                      const ts_adam_state* st, const ts_optimizer* opt, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || sh_degree < 0 || sh_degree > TS_MAX_SH_DEGREE || !opt || opt->step < 1 || !st)
        return fail(TS_EINVAL, "ts_optimizer_step: bad size, degree, step or null settings");
    if (N == 0) return TS_OK;
    if (!v || !a || !b || !sh || !o || !sigma || !gv || !go || !gsigma || !gsh || !st->m_v ||
        !st->s_v || !st->m_a || !st->s_a || !st->m_b || !st->s_b || !st->m_sh || !st->s_sh)
        return fail(TS_EINVAL, "ts_optimizer_step: null pointer");
    const float bc1 = (float)(1.0 - pow((double)opt->beta1, opt->step));
    const float bc2 = (float)(1.0 - pow((double)opt->beta2, opt->step));
    const int nsh = 3 * (sh_degree + 1) * (sh_degree + 1);
    float* const state[8] = {st->m_v, st->s_v, st->m_a, st->s_a, st->m_b, st->s_b, st->m_sh,
                             st->s_sh};
    const float lr[5] = {opt->lr_v, opt->lr_opacity, opt->lr_sigma, opt->lr_sh_dc,
                         opt->lr_sh_rest};
    ts::launch_optimizer(v, a, b, sh, o, sigma, nsh, N, gv, go, gsigma, gsh, state, lr,
                         opt->beta_opacity, opt->beta_size, opt->beta1, opt->beta2, bc1, bc2,
                         opt->eps, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_optimizer_step");
}

int ts_project_backward_adam(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                             int64_t N, const ts_proj* proj, const ts_camera* cam,
                             const ts_config* cfg, const ts_adam_state* st,
                             const ts_optimizer* opt, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || N > 0xffffffffll) return fail(TS_EINVAL, "ts_project_backward_adam: N out of range");
    if (!cam_ok(cam)) return fail(TS_EINVAL, "ts_project_backward_adam: bad camera");
    if (!cfg_ok(cfg)) return fail(TS_EINVAL, "ts_project_backward_adam: bad config");
    if (!opt || opt->step < 1 || !st)
        return fail(TS_EINVAL, "ts_project_backward_adam: bad step or null settings");
    if (N == 0) {
        if (proj) g2d_mark(proj->g2d, false);
        return TS_OK;
    }
    if (!proj_ok(proj) || !proj->cgrad || !v || !a || !b || !sh || !o || !sigma || !st->m_v ||
        !st->s_v || !st->m_a || !st->s_a || !st->m_b || !st->s_b || !st->m_sh || !st->s_sh)
        return fail(TS_EINVAL, "ts_project_backward_adam: null pointer");
    const float bc1 = (float)(1.0 - pow((double)opt->beta1, opt->step));
    const float bc2 = (float)(1.0 - pow((double)opt->beta2, opt->step));
    float* const state[8] = {st->m_v, st->s_v, st->m_a, st->s_a, st->m_b, st->s_b, st->m_sh,
                             st->s_sh};
    const float lr[5] = {opt->lr_v, opt->lr_opacity, opt->lr_sigma, opt->lr_sh_dc,
                         opt->lr_sh_rest};
    ts::launch_backproject_adam(v, a, b, sh, o, sigma, proj->cgrad, N, to_cam(cam), to_cfg(cfg),
                                proj->rect, proj->ntiles, proj->g2d, state, lr,
                                opt->beta_opacity, opt->beta_size, opt->beta1, opt->beta2, bc1,
                                bc2, opt->eps, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ts_project_backward_adam");
    g2d_mark(proj->g2d, false);
    return TS_OK;
}

size_t ts_densify_workspace_bytes(int64_t N) { return ts::densify_workspace_bytes(N < 0 ? 0 : N); }

int ts_densify_select(const float* o, const float* sigma, int64_t N, int mode, double k_expected,
                      const float* u, uint8_t* sel, void* ws, size_t ws_bytes, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || N > 0xffffffffll || (mode != TS_DENSIFY_OPACITY && mode != TS_DENSIFY_INV_SIGMA) ||
        !(k_expected >= 0.0) || k_expected > 1e300)
        return fail(TS_EINVAL, "ts_densify_select: bad size, mode or expected count");
    if (N == 0) return TS_OK;
    if (!o || !sigma || !u || !sel || !ws) return fail(TS_EINVAL, "ts_densify_select: null pointer");
    if (ws_bytes < ts::densify_workspace_bytes(N))
        return fail(TS_EWORKSPACE, "ts_densify_select: workspace too small");
    ts::launch_densify_select(o, sigma, N, mode, k_expected, u, sel, ws, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TS_OK : hip_fail(e, "ts_densify_select");
}

int ts_densify_subdivide(float* v, float* o, float* sigma, float* sh, int sh_degree, int64_t N,
                         int64_t capacity, const uint8_t* sel, void* ws, size_t ws_bytes,
                         uint32_t* d_count, uint32_t* h_count, hipStream_t stream)
{
    g_msg[0] = 0;
    if (N < 0 || capacity < N || capacity > 0xffffffffll || sh_degree < 0 ||
        sh_degree > TS_MAX_SH_DEGREE)
        return fail(TS_EINVAL, "ts_densify_subdivide: bad size, capacity or degree");
    if (!d_count || (N > 0 && (!v || !o || !sigma || !sh || !sel || !ws)))
        return fail(TS_EINVAL, "ts_densify_subdivide: null pointer");
    if (N > 0 && ws_bytes < ts::densify_workspace_bytes(N))
        return fail(TS_EWORKSPACE, "ts_densify_subdivide: workspace too small");
    if (N == 0) {
        ts::launch_fill_u32(d_count, 1, 0u, stream);
        ts::launch_fill_u32(d_count + 1, 1, 0u, stream);
    } else {
        const int nsh = 3 * (sh_degree + 1) * (sh_degree + 1);
        ts::launch_densify_subdivide(v, o, sigma, sh, nsh, N, capacity, sel, ws, d_count, stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ts_densify_subdivide");
    if (h_count) {
        e = hipMemcpyAsync(h_count, d_count, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "ts_densify_subdivide");
        if (h_count[1] != 0u)
            return fail(TS_ECAPACITY, "ts_densify_subdivide: subdivided soup exceeds capacity");
    }
    return TS_OK;
}

}  // extern "C"
