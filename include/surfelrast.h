/*
 * surfelrast.h - C ABI of the MI355X surfel (2D Gaussian) rasterizer used by
 * object-centric 2D Gaussian splatting: projection and tile binning,
 * front-to-back compositing forward and backward, the masked background
 * loss on accumulated alpha (Eq. 1) with the masked photometric L1 (Eq. 2),
 * and the occlusion-aware pruning statistics (Section 4.3).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the parameter name ends in _host.
 *     The caller allocates and owns every buffer; the library keeps no
 *     pointer after a call returns and allocates no device memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it: none synchronises, so a sequence of calls can be
 *     captured into a HIP graph.
 *   - Every call that enqueues device work takes a context (sr_create): the
 *     device it runs on and that device's status word.  Calls made while
 *     another device is current return SR_ERR_STATE.
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid call returns SR_ERR_ARG (or SR_ERR_UNSUPPORTED) and leaves the
 *     message in sr_last_error().  A HIP launch failure returns SR_ERR_HIP.
 *     Data-dependent failures (instance capacity exceeded) cannot be returned
 *     without a synchronisation: sr_bin_and_sort records them in the
 *     context's device status word, every later compositing call of the
 *     context sees the word and flags its outputs instead of computing them
 *     (per-pixel outputs and losses NaN, no gradients, no statistics, an
 *     empty prune mask), and the caller reads the word with sr_read_status
 *     after the step or graph replay.  The word stays set until
 *     sr_read_status (clear != 0) or sr_clear_status resets it.
 *   - Surfel parameters (Section 3.1: position, shape, appearance), N surfels:
 *       means  [N,3]  centre mu in world space
 *       scales [N,2]  tangent scales (s_u, s_v) > 0, already activated
 *       quats  [N,4]  rotation quaternion (w,x,y,z), any non-zero norm
 *       opac   [N]    opacity o in (0,1], already activated
 *       sh     [N,sh_stride,3] real spherical-harmonic colour coefficients
 *     all float32, contiguous.
 *   - Views: V cameras with packed outputs.  View v's pixels occupy
 *     [pix_offset, pix_offset + width*height) of every per-pixel output;
 *     multi-channel outputs (colour, normal) are planar per view:
 *     out[3*pix_offset + ch*width*height + y*width + x].
 *     Tiles are numbered globally: view v owns ids [tile_offset,
 *     tile_offset + tiles_x*tiles_y), row-major inside the view.  Tiles are
 *     binned in groups of SR_TILE_GROUP x SR_TILE_GROUP, numbered the same
 *     way from group_offset with groups_x groups per row.
 */
#ifndef SURFELRAST_H
#define SURFELRAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sr_status;
#define SR_OK 0
#define SR_ERR_ARG (-1)
#define SR_ERR_CAPACITY (-2)
#define SR_ERR_HIP (-3)
#define SR_ERR_UNSUPPORTED (-4)
#define SR_ERR_STATE (-5)

/* Bits of the device status word. */
#define SR_STATUS_CAPACITY 1u   /* a binning needed more instances than its capacity */

/* A context: the HIP device a sequence of calls runs on and that device's
 * status word (16 bytes of device memory, allocated by sr_create). */
typedef struct sr_ctx sr_ctx;

/* Pinhole camera with OpenCV axes (x right, y down, z forward); pixel (i,j)
 * is sampled at (i+0.5, j+0.5).  128 bytes; the device copy passed as
 * cams_dev must be a byte copy of the host array after sr_layout_views. */
typedef struct sr_camera {
    float viewmat[12];   /* world->camera [R|t], row-major 3x4            */
    float fx, fy, cx, cy;
    float campos[3];     /* camera centre (colour view direction)         */
    float znear;         /* surfels with centre depth <= znear are culled */
    float bg[3];         /* background colour added with the final T      */
    int32_t width, height;
    int32_t tiles_x, tiles_y; /* filled by sr_layout_views                */
    int32_t tile_offset;      /* filled by sr_layout_views                */
    int64_t pix_offset;       /* filled by sr_layout_views                */
    int32_t group_offset;     /* filled by sr_layout_views                */
    int32_t groups_x;         /* filled by sr_layout_views                */
} sr_camera;

/* Renderer configuration. */
typedef struct sr_config {
    int32_t tile_w, tile_h;   /* tile shape; see sr_tile_supported()          */
    int32_t sh_degree;        /* 0..3                                         */
    int32_t sh_stride;        /* coefficients stored per surfel, >= (deg+1)^2 */
    float alpha_min;          /* alpha cutoff, float32(1/255)                 */
    float alpha_max;          /* alpha clamp, float32(0.99)                   */
    float t_min;              /* transmittance stop, float32(1e-4)            */
    uint32_t flags;           /* SR_FLAG_*                                    */
    int32_t bwd_batch;        /* records staged per LDS batch by the backward
                                 compositing (sr_render_backward and the
                                 training steps): 32, 64, 128 or 256, at most
                                 the tile's pixel count; 0 picks
                                 min(128, tile pixels).  A tuning knob: the
                                 gradients are the same up to summation order */
} sr_config;

/* sr_render_forward / sr_prune_contrib: add to the statistics instead of
 * overwriting them (accumulation across views and calls). */
#define SR_FLAG_ACCUMULATE 1u
/* sr_backward_project: consume only the records marked by the compositing
 * backward (bit 31 of tiles_touched, set through grad_marks of
 * sr_backward_raster / sr_train_step_raster), and clear the marks.  Every
 * compositing backward since the last sr_backward_project must then have
 * been given the marks (records it added to without marking would be left
 * in grad_rec); marks are lost when sr_preprocess rewrites tiles_touched,
 * so grad_rec is consumed before the next projection. */
#define SR_FLAG_MARKED_GRADIENTS 2u

/* Per-record float counts of the intermediate buffers. */
#define SR_GEOM_STRIDE 16   /* geometry record per (view, surfel)          */
#define SR_APP_STRIDE 8     /* appearance record per (view, surfel)        */
#define SR_GRAD_STRIDE 24   /* gradient accumulator per (view, surfel)     */

/* Device counters written by sr_bin_and_sort (uint32 [4]):
 *   [0] visible (view, surfel) pairs   [1] instances required
 *   [2] instances stored (min of [1] and the capacity)
 *   [3] status: 0 ok, 1 instance capacity exceeded (outputs invalid). */
#define SR_COUNTERS 4

/* Tiles per side of a binning group, and the surfel-id bits of a sorted
 * instance value (the remaining 8 bits hold the group sub-rectangle). */
#define SR_TILE_GROUP 4
#define SR_INST_ID_BITS 24

const char *sr_last_error(void);
int32_t sr_version(void);

/* sr_create: a context on HIP device `device` (its status word zeroed);
 * the only allocation the library makes.  Host-synchronous.  Errors:
 * SR_ERR_ARG (NULL out pointer, no such device), SR_ERR_HIP.
 * sr_destroy: frees it (NULL is a no-op); the caller must not destroy a
 * context while work that uses it is still queued. */
sr_status sr_create(sr_ctx **ctx_out_host, int32_t device);
sr_status sr_destroy(sr_ctx *ctx);

/* Reads the status word after the work queued on `stream`: synchronises
 * the stream, writes the SR_STATUS_* bits to *status_bits_host and the
 * largest instance count any failed binning needed to *needed_capacity_host
 * (either may be NULL), and with clear != 0 resets the word.  Returns
 * SR_OK when no bit is set, SR_ERR_CAPACITY (with a message) when the
 * capacity bit is. */
sr_status sr_read_status(sr_ctx *ctx, void *stream, int32_t clear, uint32_t *status_bits_host,
                         uint64_t *needed_capacity_host);
/* Enqueues a reset of the status word on `stream` (a kernel, so it can be
 * captured in a HIP graph before the steps it guards). */
sr_status sr_clear_status(sr_ctx *ctx, void *stream);
/* 1 if the tile shape is compiled in, else 0. */
int32_t sr_tile_supported(int32_t tile_w, int32_t tile_h);

/* 1 if the backward compositing is compiled with `batch` records per LDS
 * batch for this tile shape (batch 0: the default, min(128, pixels)), else 0.
 * Host only; no error is recorded. */
int32_t sr_bwd_batch_supported(int32_t tile_w, int32_t tile_h, int32_t batch);

/* Host only.  Fills tiles_x, tiles_y, tile_offset, pix_offset,
 * group_offset and groups_x of the V cameras for the given tile shape and
 * returns the total pixel and tile counts.  Error: SR_ERR_ARG for V < 0, a
 * non-positive size or tile. */
sr_status sr_layout_views(sr_camera *cams_host, int32_t V, int32_t tile_w, int32_t tile_h,
                          int64_t *total_pixels_host, int32_t *total_tiles_host);

/* Projection and per-tile bounding boxes (Section 4.3: every Gaussian inside
 * the frustum is projected to the image and assigned the pixels it can
 * contribute to; one outside is disqualified).
 * For every (view v, surfel g), record index r = v*N + g:
 *   geom  [V*N, 16]  inverse splat homography, centre, opacity, depth row
 *   app   [V*N, 8]   colour, camera-space normal and the pixel rectangle
 *                    packed as two uint32 (x_lo | x_hi << 16, y_lo |
 *                    y_hi << 16; the compositing skips an entry for a
 *                    64-pixel wave whose pixels its rectangle misses)
 *                    (NULL: skip shading, e.g. for the pruning pass; sh may
 *                    then be NULL)
 *   rect  [V*N, 4]   uint16 pixel rectangle [x_lo, x_hi, y_lo, y_hi]
 *   tiles_touched [V*N] number of tiles of the rectangle (0 when culled)
 *   depth_key [V*N]  bits of float32(centre depth); 0xFFFFFFFF when culled
 *   in_frustum [N]   1 if not culled in some view (NULL to skip); with
 *                    SR_FLAG_ACCUMULATE only set, never cleared (OR over
 *                    calls)
 * Culling, rectangle and depth key are evaluated in float64 in a fixed
 * operation order, so they are reproducible bit for bit. */
sr_status sr_preprocess(sr_ctx *ctx, const sr_config *cfg, int32_t N, const float *means, const float *scales,
                        const float *quats, const float *opac, const float *sh,
                        int32_t V, const sr_camera *cams_host, const sr_camera *cams_dev,
                        float *geom, float *app, uint16_t *rect, uint32_t *tiles_touched,
                        uint32_t *depth_key, uint8_t *in_frustum, void *stream);

/* Bytes of workspace sr_bin_and_sort needs for N surfels, V views and an
 * instance capacity (instances are (view, tile group, surfel) triples). */
sr_status sr_bin_workspace_size(int32_t N, int32_t V, uint32_t inst_capacity, size_t *bytes_host);

/* Bytes of one workspace that serves every call of a training step over
 * these views that takes one (sr_bin_and_sort with this capacity,
 * sr_background_loss, sr_regularizer_loss, sr_ssim_loss with gradients,
 * sr_tile_order, sr_compact_surfels): the largest of their sizes.  Each
 * call is done with its workspace when its work on the stream ends, so
 * calls on one stream may share it. */
sr_status sr_workspace_size(const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                            uint32_t inst_capacity, size_t *bytes_host);

/* Duplicate-key generation, sort and per-tile ranges (Section 4.3: each
 * pixel blends its assigned Gaussians front to back).  Tiles are binned in
 * groups of SR_TILE_GROUP x SR_TILE_GROUP: one instance per (group, surfel)
 * whose tile rectangle meets the group, sorted by the 64-bit key (global
 * group id << 32 | depth key), equal keys by surfel id:
 *   vals   [inst_capacity] surfel id | sub << 24 of each sorted instance,
 *          sub = x_lo | x_hi << 2 | y_lo << 4 | y_hi << 6: the surfel's
 *          tile rectangle clipped to the group, in tile coordinates within
 *          the group (N must stay below 2^SR_INST_ID_BITS)
 *   keys64 [inst_capacity] the sorted keys (NULL to skip)
 *   ranges [2*T]  per global tile, [start, end) of its group's run ([0,0)
 *          if empty); the tile's own front-to-back list is the entries of
 *          that run whose sub-rectangle contains the tile
 *   counters [4]  see SR_COUNTERS
 * When the instances exceed inst_capacity the first inst_capacity of them
 * (in depth order) are sorted, counters[3] is 1 and the context's status
 * word gets SR_STATUS_CAPACITY and the count: later compositing calls of
 * the context flag their outputs.  inst_capacity 0 with vals NULL is a
 * count-only call: counters [0..1] and empty ranges, nothing emitted, the
 * status word untouched (capacity planning).
 * The depth part of the key is sorted once per visible (view, surfel)
 * before duplication; the group part by a stable LSD radix sort after it.
 * Tile-list positions used elsewhere (n_contrib, median_contrib) are
 * positions in the group run. */
sr_status sr_bin_and_sort(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                          const sr_camera *cams_dev, const uint16_t *rect, const uint32_t *tiles_touched,
                          const uint32_t *depth_key, void *workspace, size_t ws_bytes,
                          uint32_t inst_capacity, uint32_t *vals, uint64_t *keys64, uint32_t *ranges,
                          uint32_t *counters, void *stream);

/* Front-to-back alpha compositing of every view (one launch for all V
 * views).  Per pixel: colour [3P] (+ T_final * bg), alpha [P] = 1 - T_final,
 * depth [P] = sum w z, normal [3P] = sum w n, dist [P] = sum_ij w_i w_j
 * (z_i - z_j)^2, T_final [P], n_contrib [P] (position + 1 of the last
 * blended entry in the run of the pixel's tile group).  Occlusion
 * statistics of sr_prune_contrib gathered in the same pass (Section 4.3: the
 * renderer records which Gaussians the colour accumulation used), optional:
 * hits [N] alone counts the blended pixels of every surfel (hits[g] = 0 <=>
 * never blended, the pruning criterion at tau = alpha_min); hits with
 * max_alpha and max_weight [N] (both or neither) also takes the maxima;
 * cleared first unless cfg->flags has SR_FLAG_ACCUMULATE; maxima without
 * hits are an argument error.  Median depth (the 2DGS surface depth, an alternative to
 * depth/alpha in the normal consistency term of Eq. 3), optional: when
 * median_depth [P] and median_contrib [P] are not NULL (both or neither),
 * median_depth = z of the last blended entry whose transmittance before it
 * is above 1/2 (0 when no entry blends), median_contrib = that entry's
 * index + 1 in the tile list (0 when none); sr_backward_raster takes
 * median_contrib to route dL/d(median depth).  tile_order [T] / tile_cost
 * [T], optional: as for sr_train_step_raster (launch order; each tile's
 * largest n_contrib, which orders this step's sr_backward_raster through
 * sr_tile_order).  All other outputs except the statistics are required. */
sr_status sr_render_forward(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                            const sr_camera *cams_dev, const float *geom, const float *app,
                            const uint32_t *vals, const uint32_t *ranges,
                            float *color, float *alpha, float *depth, float *normal, float *dist,
                            float *T_final, uint32_t *n_contrib,
                            uint32_t *hits, float *max_alpha, float *max_weight,
                            float *median_depth, uint32_t *median_contrib,
                            const uint32_t *tile_order, uint32_t *tile_cost, void *stream);

/* Gradient of a loss through the compositing and the projection (Section
 * 3.1: position, shape and appearance are updated by backpropagation).
 * Recomputes the forward back to front from T_final and n_contrib.
 * dL_d* are the upstream gradients of the five forward outputs (any may be
 * NULL = zero); dL_dmedian [P] that of the median depth, which needs the
 * median_contrib [P] of the same forward (both NULL without it).  The
 * median depth is the depth of one entry, so its gradient reaches only that
 * entry's depth (the choice of the entry is piecewise constant).
 * grad_rec [V*N, 24] is scratch (cleared by the call, and left zero).
 * The parameter gradients are ACCUMULATED (+=) into g_means [N,3],
 * g_scales [N,2], g_quats [N,4], g_opac [N], g_sh [N,sh_stride,3]. */
sr_status sr_render_backward(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                             const sr_camera *cams_dev, const float *means, const float *scales,
                             const float *quats, const float *opac, const float *sh,
                             const float *geom, const float *app, const uint32_t *vals,
                             const uint32_t *ranges, const float *alpha, const float *depth,
                             const float *dist, const float *T_final, const uint32_t *n_contrib,
                             const float *dL_dcolor, const float *dL_dalpha, const float *dL_ddepth,
                             const float *dL_dnormal, const float *dL_ddist,
                             const uint32_t *median_contrib, const float *dL_dmedian, float *grad_rec,
                             float *g_means, float *g_scales, float *g_quats, float *g_opac,
                             float *g_sh, void *stream);

/* The two halves of sr_render_backward, one kernel each.
 * sr_backward_raster: the compositing backward only; ADDS the per-record
 * gradients to grad_rec [V*N, 24], which must hold zeros on entry (as left
 * by sr_backward_project or a fresh zeroed buffer).  tile_order [T],
 * optional: launch order as for sr_train_step_raster (sr_tile_order of the
 * tile costs the same step's sr_render_forward recorded).
 * grad_marks [V*N], optional: the tiles_touched array of the same
 * sr_preprocess; bit 31 of every record given a non-zero gradient is set
 * (atomic OR; the counts below it are untouched).
 * sr_backward_project: chains grad_rec to the parameter gradients (+=),
 * summed over the views, and zeroes every grad_rec record it consumed, so
 * the buffer is ready for the next step.  tiles_touched (from
 * sr_preprocess) lets it skip culled records; NULL scans every record.
 * With SR_FLAG_MARKED_GRADIENTS in cfg->flags it reads only the records
 * whose bit 31 is set and clears that bit: records that received no
 * gradient (visible but never blended: most of an object's interior) are
 * not read at all.
 * Density-control statistic (the 2DGS adaptive density control kept by
 * Section 5.1), optional: for every record not culled, densify_count[g] += 1
 * and densify_grad[g] += |dL/d delta|_2, the gradient of the loss with
 * respect to a translation delta of the splat in screen space (pixels; the
 * splat evaluated at x - delta, surface and low-pass alike), computed from
 * the record's gradients as (dL/d low-pass centre) - (A, B) . dL/dC' for
 * w = A dx + B dy + C'.  densify_grad [N] float, densify_count [N] uint32,
 * both accumulated (+=); either may be NULL; they need tiles_touched. */
sr_status sr_backward_raster(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                             const sr_camera *cams_dev, const float *geom, const float *app,
                             const uint32_t *vals, const uint32_t *ranges, const float *alpha,
                             const float *depth, const float *dist, const float *T_final,
                             const uint32_t *n_contrib, const float *dL_dcolor, const float *dL_dalpha,
                             const float *dL_ddepth, const float *dL_dnormal, const float *dL_ddist,
                             const uint32_t *median_contrib, const float *dL_dmedian,
                             float *grad_rec, uint32_t *grad_marks, const uint32_t *tile_order, void *stream);
sr_status sr_backward_project(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                              const sr_camera *cams_dev, const float *means, const float *scales,
                              const float *quats, const float *sh, const float *geom, const float *app,
                              uint32_t *tiles_touched, float *grad_rec, float *g_means,
                              float *g_scales, float *g_quats, float *g_opac, float *g_sh,
                              float *densify_grad, uint32_t *densify_count, void *stream);

/* Bytes of workspace sr_background_loss needs for these views. */
sr_status sr_loss_workspace_size(int32_t V, const sr_camera *cams_host, size_t *bytes_host);

/* Masked losses of every view (Eq. 1 and the L1 part of Eq. 2), loss [2V+1]:
 *   loss[v]     = L_b,v = (1/(H W)) sum A (1 - M)
 *   loss[V + v] = L1_v  = (1/(3 H W)) sum |M C - M I|     (0 without color)
 *   loss[2V]    = L = (1/V) sum_v (w_c L1_v + gamma L_b,v)
 * and the gradients of L:
 *   dL_dalpha [P] = gamma (1 - M) / (H W V)                (overwritten)
 *   dL_dcolor [3P] = w_c M sign(C - I) / (3 H W V)         (overwritten)
 * mask [P] uint8 in {0,1}.  color, target and dL_dcolor may all be NULL.
 * The per-view sums use a fixed reduction order (deterministic). */
sr_status sr_background_loss(sr_ctx *ctx, int32_t V, const sr_camera *cams_host, const sr_camera *cams_dev,
                             const float *alpha, const uint8_t *mask, const float *color,
                             const float *target, float gamma, float w_c, void *workspace,
                             size_t ws_bytes, float *loss, float *dL_dalpha, float *dL_dcolor,
                             void *stream);

/* The 2DGS regularisers of the total loss (Eq. 3: alpha L_d + beta L_n, not
 * masked), from the rendered alpha, depth, normal and distortion of every
 * view, with the readings
 *   L_d,v = (1/(H W)) sum_p dist(p)
 *   P(p)  = s(p) ((i + 0.5 - cx)/fx, (j + 0.5 - cy)/fy, 1), s = depth/alpha
 *           where alpha > 0, else 0 (camera-space point of pixel (i, j));
 *           with median [P] not NULL, s = median (the median depth of
 *           sr_render_forward) instead
 *   N_d(p) = n / max(|n|, 1e-12), n = (P(i,j+1) - P(i,j-1)) x (P(i+1,j) -
 *           P(i-1,j)); 0 on the one-pixel border
 *   L_n,v = (1/(H W)) sum_p (alpha(p) - normal(p) . N_d(p))
 * loss [2V+1]: loss[v] = L_d,v, loss[V+v] = L_n,v,
 *   loss[2V] = (1/V) sum_v (w_dist L_d,v + w_normal L_n,v);
 * gradients of loss[2V] (N_d is differentiated, so depth and alpha also get
 * the gradient through the neighbours' depth normals):
 *   dL_dalpha [P]  ADDED to (composes with sr_background_loss, which writes it)
 *   dL_ddepth [P], dL_dnormal [3P], dL_ddist [P]  overwritten
 *   dL_dmedian [P]  overwritten; required exactly when median is given
 *                   (dL_ddepth is then zero: the surface depth no longer
 *                   depends on depth)
 * Feed all of them to sr_backward_raster.  workspace: sr_loss_workspace_size
 * bytes.  Per-view sums in a fixed order (deterministic). */
sr_status sr_regularizer_loss(sr_ctx *ctx, int32_t V, const sr_camera *cams_host, const sr_camera *cams_dev,
                              const float *alpha, const float *depth, const float *normal,
                              const float *dist, const float *median, float w_dist, float w_normal,
                              void *workspace, size_t ws_bytes, float *loss, float *dL_dalpha,
                              float *dL_ddepth, float *dL_dnormal, float *dL_ddist, float *dL_dmedian,
                              void *stream);

/* Bytes of workspace sr_ssim_loss needs for these views (with_grad != 0:
 * room for the gradient maps too). */
sr_status sr_ssim_workspace_size(int32_t V, const sr_camera *cams_host, int32_t with_grad,
                                 size_t *bytes_host);

/* Masked structural similarity of every view (the D-SSIM part of Eq. 2's
 * photometric loss, applied to M*R and M*I like the L1 part) and the masked
 * metrics.  Per colour channel, with x = M R and y = M I and G the 11x11
 * Gaussian window (sigma 1.5, normalised; correlation with zero padding):
 *   S(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)),
 *   mu = G*x, s_x = G*x^2 - mu_x^2, s_xy = G*(xy) - mu_x mu_y, C1 = 1e-4, C2 = 9e-4
 * out [2V+1]: out[v] = SSIM_v (mean of S over the 3 channels and H W pixels),
 *   out[V+v] = PSNR_v = -10 log10(mean (x - y)^2) (+inf when equal),
 *   out[2V] = (1/V) sum_v w_s (1 - SSIM_v)
 * dL_dcolor [3P]: the gradient of out[2V] is ADDED (compose with
 * sr_background_loss, which writes the L1 gradient); NULL computes the
 * metrics only.  Full 3DGS photometric loss: w_c = 1 - lambda for the L1 term
 * and w_s = lambda (0.2).  mask [P] uint8; planar colour like the renderer.
 * Per-view sums in a fixed order (deterministic). */
sr_status sr_ssim_loss(sr_ctx *ctx, int32_t V, const sr_camera *cams_host, const sr_camera *cams_dev,
                       const float *color, const float *target, const uint8_t *mask, float w_s,
                       void *workspace, size_t ws_bytes, float *out, float *dL_dcolor, void *stream);

/* Fused training step of the compositing, one launch for all views: per
 * tile, the forward of sr_render_forward (same outputs, same decisions;
 * the same optional statistics: hits alone, counted by the backward phase
 * from the same blend decisions, or hits with both maxima), the masked
 * L1 + background loss gradients of sr_background_loss for every pixel
 * (Eq. 1, Eq. 2; mask [P] uint8, target [3P]), and the backward of
 * sr_backward_raster, with the per-pixel state kept on chip.
 *   tile_loss [2T]  scratch: per-tile partial sums
 *   loss [2V+1]     as sr_background_loss (sums in tile order)
 *   grad_rec        as sr_backward_raster (zeros on entry; gradients added)
 *   grad_marks      optional, as sr_backward_raster
 *   tile_order [T]  optional (NULL: the default order): the tile of each
 *                   workgroup, a permutation of 0..T-1 as sr_tile_order
 *                   writes it (heaviest tiles first); results do not depend
 *                   on it (gradients up to the rounding order of float
 *                   atomics); an entry >= T leaves its workgroup idle, so an
 *                   array that is not a permutation leaves tiles unrendered
 *   tile_cost [T]   optional (NULL: not recorded): written with each tile's
 *                   cost, the largest n_contrib of its pixels (the run
 *                   positions the tile works through), for the next call's
 *                   order
 * Follow with sr_backward_project for the parameter gradients. */
sr_status sr_train_step_raster(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                               const sr_camera *cams_dev, const float *geom, const float *app,
                               const uint32_t *vals, const uint32_t *ranges, const uint8_t *mask,
                               const float *target, float gamma, float w_c, float *color, float *alpha,
                               float *depth, float *normal, float *dist, float *T_final,
                               uint32_t *n_contrib, uint32_t *hits, float *max_alpha, float *max_weight,
                               float *tile_loss, float *loss, float *grad_rec, uint32_t *grad_marks,
                               const uint32_t *tile_order, uint32_t *tile_cost, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sr_train_step_raster with the per-tile loss partials in a scratch array of
 * the library instead of tile_loss.  The array (2 floats per tile, at most
 * SR_NOALLOC_MAX_TILES tiles = 2 MiB) is a static device array, one per GPU
 * the library runs on, held until the process ends; its address is taken
 * when the context is created.  The call allocates nothing.  Views with more
 * than SR_NOALLOC_MAX_TILES tiles in total: SR_ERR_ARG.  Every call on one
 * GPU shares that GPU's array (each tile overwrites its own partials, so
 * nothing has to start at zero): calls that can overlap on one GPU (streams
 * without an ordering between them) race, and their losses are undefined.
 * Arguments, outputs and errors otherwise as sr_train_step_raster. */
#define SR_NOALLOC_MAX_TILES 262144
sr_status sr_train_step_raster_noalloc(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V,
                                       const sr_camera *cams_host, const sr_camera *cams_dev, const float *geom,
                                       const float *app, const uint32_t *vals, const uint32_t *ranges,
                                       const uint8_t *mask, const float *target, float gamma, float w_c,
                                       float *color, float *alpha, float *depth, float *normal, float *dist,
                                       float *T_final, uint32_t *n_contrib, uint32_t *hits, float *max_alpha,
                                       float *max_weight, float *loss, float *grad_rec, uint32_t *grad_marks,
                                       const uint32_t *tile_order, uint32_t *tile_cost, void *stream);

/* Dispatch order for sr_train_step_raster: the T tile ids sorted by
 * descending cost class of tile_cost [T], written to tile_order [T]; equal
 * classes keep ascending tile id.  The class of a cost c is c below 16 and
 * (e - 3) * 16 + ((c >> (e - 4)) & 15) above, e = floor(log2 c): a
 * logarithmic scale with 16 classes per octave (the order only needs to be
 * approximately longest first; one radix pass).  The per-tile
 * work of a training step varies by two orders of magnitude (tiles near a
 * camera, under large splats); launched heaviest first, no heavy tile is left
 * for the end of the grid.  The costs of one step order the next (the views
 * and, slowly, the parameters change between steps).  workspace: device
 * memory of sr_tile_order_workspace_size bytes; no host synchronisation. */
sr_status sr_tile_order_workspace_size(int32_t T, size_t *bytes_host);
sr_status sr_tile_order(sr_ctx *ctx, int32_t T, const uint32_t *tile_cost, void *workspace, size_t ws_bytes,
                        uint32_t *tile_order, void *stream);

/* Occlusion-aware pruning statistics of one binned batch of views (Section
 * 4.3), the statistics stage of sr_prune_contrib: the compositing
 * decisions of sr_render_forward without shading.  For every blended
 * (pixel, surfel) pair: hits[g] += 1, max_alpha[g] = max(., a),
 * max_weight[g] = max(., a T).  hits [N] uint32, max_alpha [N],
 * max_weight [N] float32; cleared first unless cfg->flags has
 * SR_FLAG_ACCUMULATE.  geom and rect come from sr_preprocess (app not
 * needed); with rect [V*N, 4] each 64-pixel wave skips the entries that
 * cannot reach its pixels, as sr_render_forward does (NULL: every entry is
 * evaluated; the statistics are the same up to float32 ties). */
sr_status sr_prune_stats(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                           const sr_camera *cams_dev, const float *geom, const uint16_t *rect,
                           const uint32_t *vals, const uint32_t *ranges, uint32_t *hits,
                           float *max_alpha, float *max_weight, void *stream);

/* Work accounting of the compositing (no outputs): counts[0] = pairs
 * (pixel, tile-list entry) tested before the pixel terminated, counts[1] =
 * pairs blended, counts[2] = (64-pixel wave, entry) steps taken, counts[3] =
 * those steps in which at least one pixel of the wave blends, counts[4] =
 * pairs tested up to and including each pixel's last blended entry (the
 * pairs its backward revisits); uint64 [5], overwritten.  Entries whose
 * pixel rectangle misses all pixels of a wave are skipped by that wave and
 * not counted.  The same decisions as sr_render_forward (app as given to
 * it); used to express throughput as a fraction of the VALU roofline. */
sr_status sr_render_count(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                          const sr_camera *cams_dev, const float *geom, const float *app,
                          const uint32_t *vals, const uint32_t *ranges, uint64_t *counts, void *stream);

/* The pruning pass for 3D Gaussians (Appendix B: Section 4.3's statistics
 * for 3DGS).  sr_preprocess_3d: per (view, Gaussian) the EWA projection
 * Sigma_2 = J R_v R S S^T R^T R_v^T J^T + 0.3 I (J the perspective Jacobian at
 * the centre with x/z and y/z clamped to 1.3 tan(fov/2)), the opacity-aware
 * conservative pixel rectangle of o exp(-q/2) >= alpha_min, q = d^T
 * Sigma_2^-1 d (half extents sqrt(r2 Sigma_2,xx), sqrt(r2 Sigma_2,yy), r2 =
 * 2 ln(o/alpha_min) rounded up to 2^-16), culls (near plane, opacity,
 * degenerate, empty rectangle) and the depth key, in float64 with a fixed
 * operation order; rect / tiles_touched / depth_key are laid out as for
 * sr_preprocess and feed sr_bin_and_sort unchanged.  scales [N,3] (all
 * three axes), quats [N,4], opac [N]; geom3 [V*N, 8] float32 (conic a, b, c,
 * opacity, centre x, y, ln(o/alpha_min), 0).
 * sr_prune_stats_3d: the statistics of sr_prune_stats (hits, max alpha,
 * max weight; cleared first unless SR_FLAG_ACCUMULATE) with a = min(alpha_max,
 * o exp(-q/2)), the same cutoff, clamp and termination, lists from
 * sr_bin_and_sort. */
sr_status sr_preprocess_3d(sr_ctx *ctx, const sr_config *cfg, int32_t N, const float *means, const float *scales,
                           const float *quats, const float *opac, int32_t V, const sr_camera *cams_host,
                           const sr_camera *cams_dev, float *geom3, uint16_t *rect, uint32_t *tiles_touched,
                           uint32_t *depth_key, uint8_t *in_frustum, void *stream);
sr_status sr_prune_stats_3d(sr_ctx *ctx, const sr_config *cfg, int32_t N, int32_t V, const sr_camera *cams_host,
                              const sr_camera *cams_dev, const float *geom3, const uint32_t *vals,
                              const uint32_t *ranges, uint32_t *hits, float *max_alpha, float *max_weight,
                              void *stream);

/* Stream compaction of per-surfel arrays after pruning (Section 4.3): keep
 * surfel g when prune_mask[g] == 0 and (opac == NULL or opac[g] >=
 * min_opacity); for every array a, dst[a] row j = src[a] row i for the j-th
 * kept surfel i in increasing order (stable).  n_arrays <= SR_COMPACT_MAX_ARRAYS
 * float32 arrays of widths_host[a] floats per surfel (e.g. 3 means, 2
 * scales, 4 quats, 1 opacity, K*3 SH, and the optimiser moments alike);
 * src_host / dst_host: host arrays of device pointers; dst must not alias
 * src.  n_kept: device uint32, written.  workspace: sr_compact_workspace_size
 * bytes. */
#define SR_COMPACT_MAX_ARRAYS 8
sr_status sr_compact_workspace_size(int32_t N, size_t *bytes_host);
sr_status sr_compact_surfels(sr_ctx *ctx, int32_t N, const uint8_t *prune_mask, const float *opac, float min_opacity,
                             int32_t n_arrays, const float *const *src_host, float *const *dst_host,
                             const int32_t *widths_host, void *workspace, size_t ws_bytes,
                             uint32_t *n_kept, void *stream);

/* The whole occlusion-aware pruning pass (Section 4.3; Section 5.3 and
 * Appendix B run it over every training view of a trained model): for
 * every view, projection without shading, binning and the compositing
 * decisions, the statistics accumulated over all V views, then the mask.
 *   prim      SR_PRIM_SURFEL (2D Gaussians: scales [N,2]) or SR_PRIM_GAUSS3D
 *             (3D Gaussians: scales [N,3], the EWA path of sr_preprocess_3d)
 *   means [N,3], scales, quats [N,4], opac [N]: as sr_preprocess
 *   cams      V views laid out together by sr_layout_views (host and device
 *             copies); they are processed views_per_chunk at a time
 *             (bounding the per-view records), each chunk binned with
 *             inst_capacity instances (sr_prune_plan gives the count)
 *   workspace sr_prune_workspace_size bytes
 *   hits [N] uint32, max_alpha [N], max_weight [N] float32: the statistics
 *             of sr_prune_stats over all views; in_frustum [N] uint8: 1 if
 *             not culled in some view (NULL to skip); all cleared first
 *             unless cfg->flags has SR_FLAG_ACCUMULATE (accumulation over
 *             calls: sum, max, OR)
 *   prune_mask [N] uint8: max_alpha < tau (1 = prune; tau = alpha_min is
 *             "never blended in any view"); NULL to skip
 * Enqueued on `stream`, no synchronisation.  A chunk whose instances exceed
 * inst_capacity sets the status word; the statistics of that chunk and of
 * every later one are not taken and the mask is left all zero (prune
 * nothing): check sr_read_status. */
#define SR_PRIM_SURFEL 0
#define SR_PRIM_GAUSS3D 1
sr_status sr_prune_workspace_size(const sr_config *cfg, int32_t prim, int32_t N, int32_t V,
                                  const sr_camera *cams_host, int32_t views_per_chunk, uint32_t inst_capacity,
                                  size_t *bytes_host);
sr_status sr_prune_contrib(sr_ctx *ctx, const sr_config *cfg, int32_t prim, int32_t N, const float *means,
                           const float *scales, const float *quats, const float *opac, int32_t V,
                           const sr_camera *cams_host, const sr_camera *cams_dev, int32_t views_per_chunk,
                           float tau, uint32_t inst_capacity, void *workspace, size_t ws_bytes, uint32_t *hits,
                           float *max_alpha, float *max_weight, uint8_t *in_frustum, uint8_t *prune_mask,
                           void *stream);
/* Capacity planning for sr_prune_contrib: projects and counts the
 * instances of every chunk (count-only binning) and writes the largest
 * count to *inst_capacity_host.  SYNCHRONISES `stream` (the one pruning
 * call that does).  workspace: sr_prune_workspace_size bytes for
 * inst_capacity 0. */
sr_status sr_prune_plan(sr_ctx *ctx, const sr_config *cfg, int32_t prim, int32_t N, const float *means,
                        const float *scales, const float *quats, const float *opac, int32_t V,
                        const sr_camera *cams_host, const sr_camera *cams_dev, int32_t views_per_chunk,
                        void *workspace, size_t ws_bytes, uint32_t *inst_capacity_host, void *stream);

/* prune_mask[g] = max_alpha[g] < tau (1 = prune).  With tau = alpha_min
 * this is "never blended in any view" (Section 4.3).  While the context's
 * status word is set the mask is written all zero (prune nothing). */
sr_status sr_prune_mask(sr_ctx *ctx, int32_t N, const float *max_alpha, float tau, uint8_t *prune_mask, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SURFELRAST_H */
