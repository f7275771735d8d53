/*
 * ts.h -- C ABI of the MI355X (gfx950) triangle-splatting rasterizer.
 *
 * The library renders a soup of independent 3D triangles into an image and
 * back-propagates through it, as in "Triangle Splatting for Real-Time
 * Radiance Field Rendering" (arXiv 2505.19175):
 *   - each triangle has three vertices v_i, an opacity o, a smoothness sigma
 *     and spherical-harmonic colour coefficients                  (Sec. 3.1)
 *   - vertices are projected with a pinhole camera q = K(R v + t)  (Sec. 3.1)
 *   - each pixel p weighs a triangle by the window
 *     I(p) = ReLU(phi(p)/phi(s))^sigma, phi the 2D signed distance to the
 *     triangle and s its incentre                                  (Eq. 1)
 *   - colours are blended front to back in depth order with o*I as opacity
 *     (Sec. 3.1; the blending weight T*o of Sec. 3.2)
 *   - triangles are assigned to 16x16 pixel tiles through a tight box that
 *     drops the rim where o*I < tau_cutoff                         (Supp., "Tile assignment")
 *   - the depth order is that of the triangle centres             (Supp., "Depth sorting")
 *   - SH colour up to degree 3, 59 parameters per triangle        (Sec. 4, "Implementation details")
 * and, around that path, what a training step needs: the two window
 * alternatives the paper discusses (Sec. 3.1; Eq. 2), the pruning
 * statistics (Sec. 3.2, "Pruning"), the densification sampling and midpoint
 * subdivision (Sec. 3.2, "Densification"), the photometric loss with its
 * regularizers and Adam (Sec. 3.3).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - camera: x_c = R v + t with OpenCV axes (x right, y down, z forward);
 *     q = (fx x_c/z_c + cx, fy y_c/z_c + cy); pixel (i,j) is sampled at its
 *     centre (i+1/2, j+1/2)
 *   - a triangle is dropped if any vertex has z_c <= z_near, if its 2D
 *     inradius is below r_min, if o < alpha_min (o <= alpha_min for the
 *     sigmoid window), or if its tight box holds no pixel centre; no
 *     back-face culling
 *   - alpha = min(alpha_max, o*I); a fragment with alpha < alpha_min is
 *     skipped; one whose T(1-alpha) would fall below T_min ends the pixel
 *   - depth key = float32 of the mean camera-space z of the three vertices,
 *     ties broken by triangle index
 *   - colour = max(0, sum_k sh_k Y_k(d) + 1/2), d the unit direction from
 *     the camera centre to the triangle centroid, Y_k the real orthonormal
 *     SH basis with index l*l+l+m and no Condon-Shortley phase
 *   - outputs: rgb = sum w c + bg T_final, alpha = 1 - T_final,
 *     depth = sum w z (not normalised)
 *
 * Memory: every pointer argument except the ts_camera / ts_config structs
 * and h_count is a DEVICE pointer owned by the caller; the library never
 * allocates or frees.  Buffers are row-major and contiguous; images are
 * planar [C][H][W] float32.  All calls are asynchronous on `stream`; only
 * ts_bin_sort and ts_densify_subdivide with a non-NULL h_count synchronise
 * it.
 *
 * Errors: every entry point returns TS_OK (0) or a TS_E* code and launches
 * nothing on a validation error.  TS_EHIP wraps a failed HIP launch (the HIP
 * error string is available from ts_last_error()).  Inputs are not checked
 * for NaN/Inf.
 */
#ifndef TS_H
#define TS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TS_OK 0
#define TS_EINVAL 1      /* null pointer, negative size, bad degree, image too large */
#define TS_ECAPACITY 2   /* instance count exceeds ts_bins.capacity */
#define TS_EWORKSPACE 3  /* workspace smaller than the size query */
#define TS_EHIP 4        /* a HIP call failed */

#define TS_TILE 16               /* tile edge in pixels */
#define TS_G2D_STRIDE 16         /* floats per triangle in ts_proj.g2d */
#define TS_CGRAD_STRIDE 12       /* floats per triangle in ts_proj.cgrad */
#define TS_MAX_SH_DEGREE 3
#define TS_MAX_IMAGE_DIM 16384   /* width and height limit (int16 pixel rects) */

/* Pinhole camera (Sec. 3.1): world -> camera x_c = R v + t, R row-major. */
typedef struct ts_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} ts_camera;

/* Window functions (Sec. 3.1).  With phi the 2D signed distance (max over
 * the three edge lines, pixels, negative inside) and s the incentre:
 *   TS_WINDOW_PAPER    I = ReLU(phi(p)/phi(s))^sigma                 (Eq. 1)
 *   TS_WINDOW_SIGMOID  I = sigmoid(-phi(p)/sigma); needs o > alpha_min;
 *                      support = the triangle grown or shrunk by
 *                      sigma ln(o/alpha_min - 1) px (whole image when
 *                      alpha_min = 0)                                  (Eq. 2)
 *   TS_WINDOW_LSE      Eq. 1 with phi replaced by log sum_k exp L_k(p),
 *                      L_k the signed distance to edge k; triangles with
 *                      inradius <= ln 3 px have no inside and are culled
 * The last two are the alternatives the paper discusses and sets aside. */
#define TS_WINDOW_PAPER 0
#define TS_WINDOW_SIGMOID 1
#define TS_WINDOW_LSE 2

/* Rasterizer constants: alpha_min is the paper's tau_cutoff. */
typedef struct ts_config {
    float alpha_min;   /* cut-off: fragments with alpha < alpha_min are skipped (1/255) */
    float alpha_max;   /* opacity clamp (0.99) */
    float T_min;       /* early-termination transmittance (1e-4) */
    float z_near;      /* near plane (0.2) */
    float r_min;       /* smallest 2D inradius kept, pixels (1e-6) */
    int32_t sh_degree; /* 0..3 */
    float bg[3];       /* background colour */
    int32_t window;    /* TS_WINDOW_* (0: the paper's window) */
} ts_config;

/* Per-view projection state, N entries each, allocated by the caller.
 * Written by ts_project, read by ts_bin_sort and the renderers. */
typedef struct ts_proj {
    void* rec;          /* [N] raster records, ts_proj_record_bytes() each, 16-byte aligned */
    int16_t* rect;      /* [N][4] tight pixel box px0, px1, py0, py1 (px0 > px1: empty) */
    float* depth;       /* [N] depth key */
    uint32_t* ntiles;   /* [N] tiles covered; 0 = culled */
    float* g2d;         /* [N][TS_G2D_STRIDE] per-triangle 2D gradient accumulators:
                           the caller zero-fills it once; every ts_render_backward (or
                           ts_raster_backward followed by ts_project_backward) adds
                           into it, consumes it and leaves it zero again */
    float* cgrad;       /* [N][TS_CGRAD_STRIDE] per visible triangle, written by ts_project
                           for the backward: J[c][b] = d(sum_k sh_kc Y_k)/d dir_b at the
                           view direction (9 floats), then the channels whose colour is
                           not clamped at zero (bits 0-2 of the 10th float's bits);
                           16-byte aligned; may be NULL for forward-only use */
} ts_proj;

/* Tile lists of one view.  keys/vals/ranges are outputs of ts_bin_sort. */
typedef struct ts_bins {
    uint64_t* keys;     /* [capacity] (tile << 32) | depth bits, sorted; may be NULL */
    uint32_t* vals;     /* [capacity] triangle index of each instance, sorted */
    uint32_t* ranges;   /* [tiles][2] [start, end) of each tile in vals; (0,0) if empty */
    uint32_t* d_count;  /* [4] device counters: [0] instances M, [1] visible N_v,
                           [2] overflow flag (M > capacity), [3] tiles holding more
                           than 4096 instances */
    uint64_t capacity;  /* entries available in keys / vals */
    uint32_t* order;    /* [tiles] tiles by decreasing list length (the order in which
                           the rasterizers take them); may be NULL: natural order */
    uint16_t* blocks;   /* [capacity] per instance, bit 4 q + b: the 4x4 pixel block b of
                           8x8 quadrant q of its tile holds a pixel where the instance
                           was composited; written by ts_render_forward, read by the
                           backward to skip the blocks where it contributed nothing
                           (2 bytes per instance, not per fragment); may be NULL */
    uint32_t flags;     /* TS_BINS_SEGMENTED_SORT: depth-sort the tiles of more than 4096
                           instances with a segmented radix sort spread over many
                           workgroups (13 more launches) instead of one workgroup per
                           tile; worth setting when d_count[3] of a similar view was
                           non-zero (wide windows, dense or low-resolution views) */
} ts_bins;

#define TS_BINS_SEGMENTED_SORT 1u

/* Bytes of one raster record (the layout is private to the library). */
size_t ts_proj_record_bytes(void);

/* Tiles of a width x height image: ceil(W/16) * ceil(H/16). */
int32_t ts_num_tiles(int32_t width, int32_t height);

/* Workspace bytes ts_bin_sort needs for N triangles, `capacity` instances
 * and `num_tiles` tiles. */
size_t ts_bin_sort_workspace_bytes(int64_t N, uint64_t capacity, int32_t num_tiles);

/*
 * Projection, culling, window set-up and SH colour (Sec. 3.1; Supp. "Tile
 * assignment"), one thread per triangle, set-up in FP64.
 *   v      [N][3][3] vertices (world)        o     [N] opacity in (0,1]
 *   sigma  [N] window smoothness > 0         sh    [N][(deg+1)^2][3] SH coefficients
 * Writes every field of *out for all N triangles (records only for visible
 * ones).  N = 0 is valid and launches nothing.
 */
int ts_project(const float* v, const float* o, const float* sigma, const float* sh, int64_t N,
               const ts_camera* cam, const ts_config* cfg, const ts_proj* out,
               hipStream_t stream);

/*
 * Tile binning and depth ordering (Supp. "Tile assignment", "Depth
 * sorting"): each visible triangle emits one instance per 16x16 tile of its
 * tight box; instances are stably ordered by (tile, depth key, triangle
 * index) and ranges[t] gives tile t's run.  Device counting and radix
 * sorts, no host round trip unless h_count is non-NULL.
 *   ws/ws_bytes  workspace of ts_bin_sort_workspace_bytes(N, capacity, tiles)
 *   h_count      optional host uint32_t[2]: receives (M, N_v); the call then
 *                synchronises `stream` (and may size later launches exactly).
 *                With h_count == NULL the launches are sized by N and
 *                capacity and read M from out->d_count on the device.
 * Returns TS_ECAPACITY when M > capacity and h_count is non-NULL (M is left
 * in h_count[0] and d_count[0]; the ranges and order then describe valid,
 * possibly empty, runs); with h_count == NULL an overflow sets d_count[2]
 * and the lists hold `capacity` of the M instances (which ones depends on
 * the grouping path), each tile's run in (depth, index) order.
 */
int ts_bin_sort(const ts_proj* proj, int64_t N, const ts_camera* cam, void* ws, size_t ws_bytes,
                const ts_bins* out, uint32_t* h_count, hipStream_t stream);

/*
 * ts_bin_sort without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as ts_bin_sort; the workspace is a fixed device array of
 * TS_NOALLOC_SCRATCH_BYTES inside the library (one copy per GPU, held until
 * the process ends).  The call allocates nothing: its first call on a
 * device, with that device current, resolves the array's address once
 * (hipGetSymbolAddress; make that first call outside a graph capture).
 *   Returns TS_EWORKSPACE, launching nothing, when
 *   ts_bin_sort_workspace_bytes(N, out->capacity, tiles) exceeds the array
 *   (about 3M instances at 3M triangles and 3600 tiles).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero; each call writes
 * what it reads.
 */
#define TS_NOALLOC_SCRATCH_BYTES (64u << 20)

int ts_bin_sort_noalloc(const ts_proj* proj, int64_t N, const ts_camera* cam, const ts_bins* out,
                        uint32_t* h_count, hipStream_t stream);

/*
 * Forward compositing (Eq. 1; Sec. 3.1): one 256-thread workgroup per tile,
 * records staged through LDS, per-pixel FP64 edge functions and FP32
 * blending, wavefront-ballot early termination.
 * Outputs (device, [H][W] unless noted): rgb [3][H][W], alpha, depth,
 * T_final (transmittance left), last (number of list entries of the pixel's
 * tile up to and including its last composited fragment; backward state).
 * When bins->blocks is set it also receives, per list entry, the 4x4 blocks
 * where that entry was composited (entries after a tile's last composited
 * one may be left unwritten; the backward never reads them).
 */
int ts_render_forward(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                      const ts_config* cfg, float* rgb, float* alpha, float* depth,
                      float* T_final, uint32_t* last, hipStream_t stream);

/*
 * Per-triangle pruning statistics (Sec. 3.2, "Pruning": a triangle whose
 * largest blending weight T*o over the training views stays below a
 * threshold is pruned, and so is one rendered with more than one pixel in
 * fewer than two views).  Device arrays of N entries, caller-initialised:
 *   max_weight  max(existing value, largest T*o at a fragment of the triangle
 *               that is composited; T the transmittance in front of it);
 *               non-negative, zero-fill for a fresh count
 *   pixels      += the number of pixels where the triangle is composited
 */
typedef struct ts_prune_stats {
    float* max_weight;
    uint32_t* pixels;
} ts_prune_stats;

/* ts_render_forward that also accumulates the pruning statistics of the
 * view into *stats, indexed by triangle (N entries each, N of the
 * projection).  Max and add atomics: the result does not depend on the order
 * of the tiles.  TS_EINVAL if stats or either of its arrays is NULL. */
int ts_render_forward_stats(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, const ts_prune_stats* stats,
                            hipStream_t stream);

/* After each view: views[i] += (pixels[i] > 1), then pixels[i] = 0, so views
 * counts the views that rendered triangle i with more than one pixel.  Device
 * arrays of N entries; TS_EINVAL if N < 0 or (N > 0 and either is NULL). */
int ts_prune_count_views(uint32_t* pixels, uint32_t* views, int64_t N, hipStream_t stream);

/*
 * Backward pass (end-to-end gradients, Sec. 3.3): reverse traversal of each
 * pixel's composited fragments, transmittance recovered from T_final (no
 * per-fragment state), per-wavefront reduction before atomics into
 * proj->g2d, then one thread per triangle chains the 2D gradients to the
 * vertices, opacity, sigma and SH coefficients.
 *   dL_drgb [3][H][W] required; dL_dalpha, dL_ddepth [H][W] may be NULL.
 *   T_final, last: the forward outputs of the same view; bins->blocks (if
 *   set) must be the masks that forward wrote into the same bins.
 * Gradients are overwritten (not accumulated); culled triangles get zeros.
 *   gv [N][3][3], go [N], gsigma [N], gsh [N][(deg+1)^2][3]
 */
int ts_render_backward(const float* v, const float* o, const float* sigma, const float* sh,
                       int64_t N, const ts_proj* proj, const ts_bins* bins,
                       const ts_camera* cam, const ts_config* cfg, const float* dL_drgb,
                       const float* dL_dalpha, const float* dL_ddepth, const float* T_final,
                       const uint32_t* last, float* gv, float* go, float* gsigma, float* gsh,
                       hipStream_t stream);

/*
 * The two halves of ts_render_backward, for callers that schedule them
 * separately.  ts_raster_backward accumulates the per-triangle 2D gradients
 * into proj->g2d (which must hold zeros, as the caller's zero fill and
 * every ts_project_backward leave it); ts_project_backward turns them into
 * gv, go, gsigma, gsh and re-zeroes the rows it consumed.
 * Caller obligation: call ts_project_backward (or ts_project_backward_adam)
 * on the same proj after every ts_raster_backward, before the next raster
 * backward or ts_render_backward on that g2d array.  The library keeps a
 * host-side record of g2d arrays filled and not yet consumed (up to 64 at a
 * time) and returns TS_EINVAL, launching nothing, for a raster backward on
 * one of them.
 */
int ts_raster_backward(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                       const ts_config* cfg, const float* dL_drgb, const float* dL_dalpha,
                       const float* dL_ddepth, const float* T_final, const uint32_t* last,
                       hipStream_t stream);

int ts_project_backward(const float* v, const float* sh, int64_t N, const ts_proj* proj,
                        const ts_camera* cam, const ts_config* cfg, float* gv, float* go,
                        float* gsigma, float* gsh, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Stored-fragment variant, kept to measure what the recompute backward saves:
 * the forward keeps every composited fragment (its tile-list entry, alpha
 * and the transmittance in front of it, 12 bytes) and the backward reads
 * them instead of recovering transmittance from T_final (Sec. 3.3
 * gradients; the same arithmetic as ts_render_forward / ts_raster_backward).
 * ------------------------------------------------------------------------ */

/* Workspace bytes of ts_render_forward_count for a width x height view. */
size_t ts_fragment_workspace_bytes(int32_t width, int32_t height);

/* ts_render_forward that also writes, per pixel, the number of composited
 * fragments (frag_count [H][W]) and their first slot (frag_offset [H][W], the
 * exclusive prefix sum in row-major pixel order), and F, their total, into
 * d_total[0] (device).  TS_EINVAL for a null pointer, TS_EWORKSPACE when
 * ws_bytes < ts_fragment_workspace_bytes(W, H). */
int ts_render_forward_count(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, uint32_t* frag_count,
                            uint32_t* frag_offset, uint32_t* d_total, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* ts_render_forward that stores every composited fragment of pixel p at
 * slots frag_offset[p] + 0, 1, ... in blending order (frag_offset from
 * ts_render_forward_count on the same bins): frag_entry = its index in the
 * tile's list, frag_alpha, frag_T = transmittance in front of it; arrays of
 * F entries (device). */
int ts_render_forward_store(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                            const ts_config* cfg, float* rgb, float* alpha, float* depth,
                            float* T_final, uint32_t* last, const uint32_t* frag_offset,
                            uint32_t* frag_entry, float* frag_alpha, float* frag_T,
                            hipStream_t stream);

/* ts_raster_backward reading the stored fragments (no transmittance
 * recovery); the same g2d contract as ts_raster_backward. */
int ts_raster_backward_stored(const ts_proj* proj, const ts_bins* bins, const ts_camera* cam,
                              const ts_config* cfg, const float* dL_drgb, const float* dL_dalpha,
                              const float* dL_ddepth, const float* T_final, const uint32_t* last,
                              const uint32_t* frag_count, const uint32_t* frag_offset,
                              const uint32_t* frag_entry, const float* frag_alpha,
                              const float* frag_T, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched forward rendering of several views of one resident soup (serving).
 * ------------------------------------------------------------------------ */

/* One view of a batch.  tile_offset, tiles_x and pixel_offset place the
 * view's tiles and pixels in the batch; ts_batch_layout fills them. */
typedef struct ts_view {
    ts_camera cam;
    uint32_t tile_offset;   /* first batch-wide tile id of this view */
    uint32_t tiles_x;       /* ceil(width / 16) */
    uint64_t pixel_offset;  /* first pixel of this view in the packed outputs */
} ts_view;

/* Host helper: fills tile_offset, tiles_x and pixel_offset of views[0..n)
 * (in order) and returns the batch's tile and pixel totals. */
int ts_batch_layout(ts_view* views, int32_t n, uint32_t* total_tiles, uint64_t* total_pixels);

/* Workspace bytes of ts_render_forward_batched for N triangles, up to
 * max_views views, `capacity` instances and max_tiles tiles per batch. */
size_t ts_batch_workspace_bytes(int64_t N, int32_t max_views, uint64_t capacity,
                                uint32_t max_tiles);

/*
 * Forward render of a batch of views in one fixed sequence of launches
 * whose sizes do not depend on the batch content, so the sequence can be
 * captured once in a HIP graph and replayed with new views:
 *   - one projection pass loads every triangle once and sets it up for all
 *     views of the batch (record of (view, triangle) at view * N + triangle)
 *   - one binning pass orders the instances of all views by batch-wide tile
 *   - one persistent launch drains a tile queue shared by the views, so
 *     views of different resolutions balance across the chip.
 * Arguments (device unless noted):
 *   views      [max_views] views, laid out by ts_batch_layout
 *   ctl        [2] uint32: number of views in this batch, their total tiles
 *   proj       per-entry arrays of max_views * N entries (g2d may be NULL)
 *   bins       vals / keys of `capacity` entries, ranges of max_tiles tiles;
 *              d_count[2] is set when the batch's instances exceeded capacity
 *              (the frames are then incomplete and must be rendered again)
 *   rgb        packed planar outputs: view v's [3][H][W] block starts at
 *              rgb + 3 * pixel_offset; alpha / depth: [H][W] at pixel_offset
 * The same per-pixel arithmetic as ts_render_forward: a view rendered alone
 * and inside a batch gives identical pixels.
 */
int ts_render_forward_batched(const float* v, const float* o, const float* sigma,
                              const float* sh, int64_t N, const ts_view* views,
                              const uint32_t* ctl, int32_t max_views, uint32_t max_tiles,
                              const ts_config* cfg, const ts_proj* proj, const ts_bins* bins,
                              void* ws, size_t ws_bytes, float* rgb, float* alpha, float* depth,
                              hipStream_t stream);

/* Static description of an error code. */
const char* ts_error_string(int code);

/* Message of the last failure on the calling thread ("" if none). */
const char* ts_last_error(void);

/*
 * Densification (Sec. 3.2, "Densification"; Supp.): the sampling step and
 * the midpoint subdivision that runs between renders during training.
 *
 * ts_densify_select: Bernoulli sampling.  With w_i = o_i (mode
 * TS_DENSIFY_OPACITY) or 1/sigma_i (TS_DENSIFY_INV_SIGMA; the paper
 * alternates the two from step to step), triangle i is selected iff
 *     u[i] < p_i = min(1, k_expected w_i / sum_j w_j),
 * so k_expected triangles are selected on average.  u[N] holds uniform
 * numbers in [0, 1) supplied by the caller (the library draws none).  The
 * sum is FP64 in a fixed order (reproducible); p_i and the test are FP64.
 *   o, sigma, u  device [N] float;  sel  device [N] bytes, 1 = selected
 *   ws           device workspace of ts_densify_workspace_bytes(N) bytes
 * TS_EINVAL for N < 0, a null pointer, mode out of range, or k_expected
 * negative or not finite; TS_EWORKSPACE when ws_bytes is too small.
 *
 * ts_densify_subdivide: midpoint subdivision of the selected triangles, in
 * place.  Each selected triangle (v0, v1, v2) becomes four, joining the
 * edge midpoints m01, m12, m20 (computed as (a + b) * 0.5 in FP32): the
 * centre child (m01, m12, m20) replaces it at its index and the corner
 * children (v0, m01, m20), (m01, v1, m12), (m20, m12, v2) are written at
 * N + 3r, N + 3r + 1, N + 3r + 2, r the number of selected triangles before
 * it; the corner children copy its opacity, sigma and SH row.
 *   v [capacity][3][3], o, sigma [capacity], sh [capacity][(deg+1)^2][3]:
 *                device, the first N entries the current soup
 *   sel          device [N] bytes (e.g. from ts_densify_select)
 *   d_count      device [2] uint32: [0] = N + 3 n_selected, [1] = 1 when that
 *                exceeds capacity, in which case nothing is written
 *   h_count      host [2] or NULL: with it the call waits for the stream,
 *                copies d_count and returns TS_ECAPACITY on overflow
 * The triangles of the other per-triangle arrays a caller keeps (optimizer
 * moments, for instance) are not moved: it handles them from sel and
 * d_count.
 */
#define TS_DENSIFY_OPACITY 0
#define TS_DENSIFY_INV_SIGMA 1

size_t ts_densify_workspace_bytes(int64_t N);

int ts_densify_select(const float* o, const float* sigma, int64_t N, int mode, double k_expected,
                      const float* u, uint8_t* sel, void* ws, size_t ws_bytes,
                      hipStream_t stream);

int ts_densify_subdivide(float* v, float* o, float* sigma, float* sh, int sh_degree, int64_t N,
                         int64_t capacity, const uint8_t* sel, void* ws, size_t ws_bytes,
                         uint32_t* d_count, uint32_t* h_count, hipStream_t stream);

/*
 * One training step around the renderer (Sec. 3.3, "Optimization"; the
 * loss terms the paper takes from the works it cites, and the learning
 * rates of its hyperparameter table).
 *
 * ts_image_loss: the photometric loss (1 - lambda) L1 + lambda (1 - SSIM)
 * of a rendered image against a target, and its gradient.  L1 is the mean
 * |rgb - target| over the 3 H W values; SSIM is computed per channel with an
 * 11x11 Gaussian window (standard deviation 1.5, weights summing to 1),
 * C1 = 0.01^2, C2 = 0.03^2, pixels outside the image counting as zero, and
 * averaged over the 3 H W values.
 *   rgb, target  device [3][H][W] float
 *   dL_drgb      device [3][H][W] float, overwritten with dL/drgb
 *   loss         device [2] float or NULL: mean |rgb - target|, mean SSIM
 *   ws           device workspace of ts_image_loss_workspace_bytes(W, H)
 * TS_EINVAL for a non-positive size, lambda outside [0, 1] or a null
 * pointer; TS_EWORKSPACE when ws_bytes is too small.
 *
 * ts_optimizer_step: adds the opacity loss beta_o mean(o) and the size loss
 * beta_s mean(2 / |(v1 - v0) x (v2 - v0)|) to the renderer's gradients,
 * chains them to the raw parameters (o = sigmoid(a), sigma = exp(b)) and
 * applies one bias-corrected Adam step to v, a, b and sh; o and sigma are
 * rewritten from the new a and b for the next render.
 *   v [N][3][3], a, b [N], sh [N][(deg+1)^2][3]: raw parameters (device)
 *   o, sigma [N]: their activated copies (read, then rewritten)
 *   gv, go, gsigma, gsh: the renderer's gradients w.r.t. v, o, sigma, sh
 *                (as ts_render_backward writes them); read only
 *   state: the first and second moment arrays, shaped like the parameters,
 *                zero before the first step
 *   opt: learning rates, Adam constants, loss weights and the step number
 *                t >= 1 (bias correction 1 - beta^t)
 * Degree-0 SH coefficients use lr_sh_dc, the others lr_sh_rest.
 * TS_EINVAL for N < 0, a bad degree or step, or a null pointer.
 */
typedef struct ts_adam_state {
    float *m_v, *s_v, *m_a, *s_a, *m_b, *s_b, *m_sh, *s_sh;
} ts_adam_state;

typedef struct ts_optimizer {
    float lr_v, lr_opacity, lr_sigma, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float beta_opacity, beta_size;   /* weights of the opacity and size losses */
    int32_t step;                    /* t >= 1 */
} ts_optimizer;

size_t ts_image_loss_workspace_bytes(int width, int height);

int ts_image_loss(const float* rgb, const float* target, int width, int height, float lambda,
                  float* dL_drgb, float* loss, void* ws, size_t ws_bytes, hipStream_t stream);

int ts_optimizer_step(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                      int sh_degree, int64_t N, float* gv, float* go, float* gsigma, float* gsh,
                      const ts_adam_state* state, const ts_optimizer* opt, hipStream_t stream);

/* ts_project_backward_adam: ts_project_backward followed by ts_optimizer_step
 * in one pass over the triangles (Sec. 3.3: the training step's backward and
 * Adam update).  Triangles share no parameters, so a triangle's gradient is
 * complete once its own 2D gradients are chained back; the optimizer step
 * runs on it there, and no gradient array is written or read.  For callers
 * that train and need no gradients.
 *   v [N][3][3], a, b [N], sh [N][(deg+1)^2][3]: raw parameters (device), the
 *                ones the view was rendered with; updated in place
 *   o, sigma [N]: their activated copies (read, then rewritten)
 *   proj, cam, cfg: as for ts_project_backward (after ts_raster_backward);
 *                the SH degree is cfg->sh_degree; proj->g2d is consumed
 *                (re-zeroed)
 *   state, opt: as for ts_optimizer_step
 * The result is that of the two calls: both run the same FP32 steps, so it
 * differs only where the compiler contracted an expression differently.
 * TS_EINVAL for the arguments either call rejects.
 */
int ts_project_backward_adam(float* v, float* a, float* b, float* sh, float* o, float* sigma,
                             int64_t N, const ts_proj* proj, const ts_camera* cam,
                             const ts_config* cfg, const ts_adam_state* state,
                             const ts_optimizer* opt, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TS_H */
