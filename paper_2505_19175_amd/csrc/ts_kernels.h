// ts_kernels.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ts.h"

namespace ts {

struct Cam;
struct Cfg;

// Calls L<DEG, WIN>::run(args...) for a runtime SH degree (0..3) and window
// function (TS_WINDOW_*): one kernel instantiation per pair.
template <template <int, int> class L, typename... Args>
void dispatch_deg_win(int deg, int win, Args&&... args)
{
    auto by_win = [&](auto deg_c) {
        constexpr int D = decltype(deg_c)::value;
        switch (win) {
        case TS_WINDOW_SIGMOID: L<D, TS_WINDOW_SIGMOID>::run(args...); break;
        case TS_WINDOW_LSE: L<D, TS_WINDOW_LSE>::run(args...); break;
        default: L<D, TS_WINDOW_PAPER>::run(args...); break;
        }
    };
    switch (deg) {
    case 0: by_win(std::integral_constant<int, 0>{}); break;
    case 1: by_win(std::integral_constant<int, 1>{}); break;
    case 2: by_win(std::integral_constant<int, 2>{}); break;
    default: by_win(std::integral_constant<int, 3>{}); break;
    }
}

void launch_project(const float* v, const float* o, const float* sigma, const float* sh,
                    int64_t N, const Cam& cam, const Cfg& cfg, void* rec, int16_t* rect,
                    float* depth, uint32_t* ntiles, float* cgrad, hipStream_t stream);

void launch_project_views(const float* v, const float* o, const float* sigma, const float* sh,
                          int64_t N, const ts_view* views, const uint32_t* ctl, const Cfg& cfg,
                          void* rec, int16_t* rect, float* depth, uint32_t* ntiles,
                          hipStream_t stream);

// Device copy of a batch descriptor clamped to the buffers: ctl_out[0] =
// views (<= max_views), [1] = tiles (<= max_tiles), [2] = views * per_view.
void launch_batch_ctl(const uint32_t* ctl_in, uint32_t max_views, uint32_t max_tiles,
                      int64_t per_view, uint32_t* ctl_out, hipStream_t stream);

void launch_backproject(const float* v, const float* cgrad, int64_t N, const Cam& cam,
                        const Cfg& cfg, const int16_t* rect, const uint32_t* ntiles, float* g2d,
                        float* gv, float* go, float* gsig, float* gsh, hipStream_t stream);

// p[0..n) = x (a kernel, so it can sit inside a captured graph).
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t x, hipStream_t stream);

// order[0..n) = tiles by decreasing list length, n = min(*d_tiles,
// num_tiles) or num_tiles; nothing when order is null.
void launch_tile_order(const uint32_t* ranges, int num_tiles, const uint32_t* d_tiles,
                       uint32_t* order, hipStream_t stream, uint32_t* n_long = nullptr,
                       uint32_t* n_huge = nullptr);

// Workspace carve-up of the binning stage.
struct BinWorkspace {
    uint32_t* blk;      // [nbN + 1] per-block instance counts / offsets
    uint32_t* blk_vis;  // [nbN + 1] per-block visible counts
    uint32_t* hist;     // [256][hist_stride] radix block histograms
    uint32_t* dtot;     // [256] radix digit totals
    uint32_t* tk[2];    // [capacity] tile ids (ping-pong; per-tile sort scratch after)
    uint32_t* tv[2];    // [capacity] entry ids (ping-pong; per-tile sort scratch after)
    uint32_t* tfin;     // [capacity] sorted tile ids
    uint32_t* torder;   // [num_tiles] tile order when the caller keeps none
    uint32_t* hl;       // [num_tiles] the tiles of the segmented sort
    uint32_t* cst;      // [num_tiles + 2] their chunk prefix; [num_tiles + 1] = their count
    uint32_t* ctl;      // [8] device counters: [0] sort count min(M, capacity),
                        //     [1] tiles too long for the one-wave sort
    int64_t hist_stride;
    size_t bytes;
};

BinWorkspace carve_bin_workspace(void* base, int64_t N, uint64_t capacity, int64_t num_tiles);

// Device-side binning of N entries (or *d_n <= N when d_n is set).  With
// views set, entry e belongs to view e / per_view and its tiles are offset
// by that view's tile_offset.  Returns hipSuccess or the first launch error.
hipError_t run_bin_sort(const uint32_t* ntiles, const float* depth, const int16_t* rect,
                        int64_t N, const uint32_t* d_n, const ts_view* views, int64_t per_view,
                        int tiles_x, int num_tiles, const BinWorkspace& ws, const ts_bins& out,
                        uint32_t* h_count, bool* overflow, hipStream_t stream,
                        const uint32_t* d_tiles = nullptr);

// `order` (nullable) lists the tiles in the order the workgroups take them.
void launch_raster_forward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                           const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                           int num_tiles, float* rgb, float* alpha, float* depth, float* T_final,
                           uint32_t* last, uint16_t* blocks, float* max_weight, uint32_t* pixels,
                           hipStream_t stream);

// Densification (Sec. 3.2): sampling and midpoint subdivision.
size_t densify_workspace_bytes(int64_t N);
void launch_densify_select(const float* o, const float* sigma, int64_t N, int mode, double k,
                           const float* u, uint8_t* sel, void* ws, hipStream_t stream);
void launch_densify_subdivide(float* v, float* o, float* sigma, float* sh, int nsh, int64_t N,
                              int64_t capacity, const uint8_t* sel, void* ws, uint32_t* d_out,
                              hipStream_t stream);

// Training step pieces (Sec. 3.3): image loss, regularizers, Adam.
size_t image_loss_workspace_bytes(int W, int H);
void launch_image_loss(const float* rgb, const float* target, int W, int H, float lambda,
                       float* grad, float* loss, void* ws, hipStream_t stream);
// st: m_v, s_v, m_a, s_a, m_b, s_b, m_sh, s_sh; lr: v, opacity, sigma, SH dc, SH rest.
void launch_optimizer(float* v, float* a, float* b, float* sh, float* o, float* sigma, int nsh,
                      int64_t N, const float* gv, const float* go, const float* gs,
                      const float* gsh, float* const* st, const float* lr, float beta_o,
                      float beta_s, float b1, float b2, float bc1, float bc2, float eps,
                      hipStream_t stream);

// The backward projection and the optimizer step in one pass (Adam where
// each triangle's gradient is formed); st, lr and the constants as for
// launch_optimizer.
void launch_backproject_adam(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                             const float* cgrad, int64_t N, const Cam& cam, const Cfg& cfg,
                             const int16_t* rect, const uint32_t* ntiles, float* g2d,
                             float* const* st, const float* lr, float beta_o, float beta_s,
                             float b1, float b2, float bc1, float bc2, float eps,
                             hipStream_t stream);

// views[i] += pixels[i] > 1; pixels[i] = 0.
void launch_prune_views(uint32_t* pixels, uint32_t* views, int64_t N, hipStream_t stream);

void launch_raster_forward_queue(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                                 const uint32_t* order, const ts_view* views,
                                 const uint32_t* ctl, const Cfg& cfg,
                                 uint32_t* queue, int workgroups, float* rgb, float* alpha,
                                 float* depth, hipStream_t stream);

// Stored-fragment variant (the memory form the recompute backward is
// measured against): per pixel the number of composited fragments and the
// first slot of its run; per slot the tile-list entry, alpha and the
// transmittance in front of the fragment.
struct FragStore {
    uint32_t* count;
    const uint32_t* offset;
    uint32_t* entry;
    float* alpha;
    float* T;
};

// fs == nullptr: the recompute backward (transmittance recovered from
// T_final); otherwise each pixel's fragments, alphas and transmittances are
// read from *fs (written by the forward in mode 2 on the same bins).
void launch_raster_backward(const void* rec, const uint32_t* vals, const uint32_t* ranges,
                            const uint32_t* order, const Cam& cam, const Cfg& cfg, int tiles_x,
                            int num_tiles,
                            const float* dL_drgb, const float* dL_dalpha,
                            const float* dL_ddepth, const float* T_final,
                            const uint32_t* last, const uint16_t* blocks, float* g2d,
                            hipStream_t stream, const FragStore* fs = nullptr);

// The forward of the stored-fragment variant: mode 1 writes fs.count, mode 2
// stores the fragments at fs.offset (an exclusive scan of the counts).
void launch_raster_forward_fragments(const void* rec, const uint32_t* vals,
                                     const uint32_t* ranges, const uint32_t* order,
                                     const Cam& cam, const Cfg& cfg, int tiles_x, int num_tiles,
                                     float* rgb, float* alpha, float* depth, float* T_final,
                                     uint32_t* last, uint16_t* blocks, int mode,
                                     const FragStore& fs, hipStream_t stream);

// offset[p] = sum of count[0..p), total[0] = sum of all (one pass of block
// sums, one scan of them, one pass applying them); ws of
// fragment_scan_workspace_bytes(n) bytes.
size_t fragment_scan_workspace_bytes(int64_t n);
void launch_fragment_offsets(const uint32_t* count, int64_t n, uint32_t* offset, uint32_t* total,
                             void* ws, hipStream_t stream);

}  // namespace ts
