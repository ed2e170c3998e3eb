// C ABI of the surfel rasterizer: host-side argument validation and
// dispatch to the HIP kernels.  Apart from sr_create (the context's status
// word) no entry point allocates device memory, and apart from
// sr_create/sr_read_status/sr_prune_plan none synchronises; every launch goes
// to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "launch.h"
#include "surfelrast.h"

static_assert(sizeof(sr_camera) == 128, "sr_camera must stay 128 bytes");

// A context: its device and that device's status word, uint32 [4]:
// [0] SR_STATUS_* bits, [1] the largest instance count a failed binning
// needed, [2..3] unused.
struct sr_ctx {
    int device;
    uint32_t* status;
    float* scratch;     // the device's scratch array (sr_train_step_raster_noalloc)
};

namespace {

thread_local char g_err[512] = "";

sr_status fail(sr_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

sr_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return SR_OK;
    return fail(SR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

sr_status check_cfg(const sr_config* cfg) {
    if (!cfg) return fail(SR_ERR_ARG, "cfg is NULL");
    if (!sr::tile_shape_supported(cfg->tile_w, cfg->tile_h))
        return fail(SR_ERR_UNSUPPORTED, "tile shape %dx%d is not compiled in", cfg->tile_w, cfg->tile_h);
    if (cfg->sh_degree < 0 || cfg->sh_degree > 3)
        return fail(SR_ERR_UNSUPPORTED, "sh_degree %d not in 0..3", cfg->sh_degree);
    const int K = (cfg->sh_degree + 1) * (cfg->sh_degree + 1);
    if (cfg->sh_stride < K || cfg->sh_stride > 16)
        return fail(SR_ERR_ARG, "sh_stride %d must be in [%d, 16]", cfg->sh_stride, K);
    if (!(cfg->alpha_min > 0.f && cfg->alpha_min < cfg->alpha_max && cfg->alpha_max < 1.f))
        return fail(SR_ERR_ARG, "need 0 < alpha_min < alpha_max < 1");
    if (!(cfg->t_min > 0.f && cfg->t_min < 1.f)) return fail(SR_ERR_ARG, "need 0 < t_min < 1");
    if (cfg->bwd_batch != 0 && !sr::bwd_batch_supported(cfg->tile_w, cfg->tile_h, cfg->bwd_batch))
        return fail(SR_ERR_UNSUPPORTED, "backward batch %d is not compiled in for %dx%d tiles", cfg->bwd_batch,
                    cfg->tile_w, cfg->tile_h);
    return SR_OK;
}

// Views must carry the layout sr_layout_views computes for this tile shape.
sr_status check_views(const sr_camera* cams_host, const sr_camera* cams_dev, int V, int tw, int th,
                      int64_t* total_pix, int* total_tiles, int64_t* max_hw, int* total_groups = nullptr) {
    if (V < 0) return fail(SR_ERR_ARG, "V = %d < 0", V);
    if (V > 0 && (!cams_host || !cams_dev)) return fail(SR_ERR_ARG, "cams_host and cams_dev are required");
    int64_t pix = 0, mhw = 0;
    int64_t tiles = 0, groups = 0;
    for (int v = 0; v < V; ++v) {
        const sr_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
            return fail(SR_ERR_ARG, "view %d: size %dx%d outside [1, 65535]", v, c.width, c.height);
        const int tx = (c.width + tw - 1) / tw, ty = (c.height + th - 1) / th;
        const int gx = (tx + SR_TILE_GROUP - 1) / SR_TILE_GROUP, gy = (ty + SR_TILE_GROUP - 1) / SR_TILE_GROUP;
        if (c.tiles_x != tx || c.tiles_y != ty || c.tile_offset != tiles || c.pix_offset != pix ||
            c.group_offset != groups || c.groups_x != gx)
            return fail(SR_ERR_ARG, "view %d: layout fields do not match sr_layout_views for %dx%d tiles", v, tw,
                        th);
        if (!(c.fx > 0.f && c.fy > 0.f)) return fail(SR_ERR_ARG, "view %d: focal lengths must be positive", v);
        pix += (int64_t)c.width * c.height;
        tiles += (int64_t)tx * ty;
        groups += (int64_t)gx * gy;
        if ((int64_t)c.width * c.height > mhw) mhw = (int64_t)c.width * c.height;
    }
    if (tiles > 0x7FFFFFFF) return fail(SR_ERR_ARG, "too many tiles (%lld)", (long long)tiles);
    if (total_pix) *total_pix = pix;
    if (total_tiles) *total_tiles = (int)tiles;
    if (total_groups) *total_groups = (int)groups;
    if (max_hw) *max_hw = mhw;
    return SR_OK;
}

sr_status check_nv(int N, int V) {
    if (N < 0) return fail(SR_ERR_ARG, "N = %d < 0", N);
    if ((uint64_t)N * (uint64_t)(V > 0 ? V : 0) >= 0xFFFFFFFFull)
        return fail(SR_ERR_ARG, "N*V = %llu must stay below 2^32", (unsigned long long)N * V);
    return SR_OK;
}

// The context is checked after the arguments (so argument errors are
// reported without a device), right before anything is enqueued.
sr_status check_ctx(const sr_ctx* c) {
    if (!c) return fail(SR_ERR_ARG, "ctx is NULL");
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return fail(SR_ERR_HIP, "hipGetDevice failed");
    if (d != c->device)
        return fail(SR_ERR_STATE, "context of device %d used while device %d is current", c->device, d);
    return SR_OK;
}

#define SR_TRY(x)                          \
    do {                                   \
        sr_status _s = (x);                \
        if (_s != SR_OK) return _s;        \
    } while (0)

#define SR_NEED(p)                                                  \
    do {                                                            \
        if (!(p)) return fail(SR_ERR_ARG, "%s is NULL", #p);        \
    } while (0)

}  // namespace

extern "C" {

const char* sr_last_error(void) { return g_err; }

int32_t sr_version(void) { return 4; }

sr_status sr_create(sr_ctx** ctx_out_host, int32_t device) {
    if (!ctx_out_host) return fail(SR_ERR_ARG, "ctx_out_host is NULL");
    *ctx_out_host = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(SR_ERR_ARG, "no HIP device %d (%d present)", device, n);
    int prev = 0;
    SR_TRY(hip_status(hipGetDevice(&prev), "hipGetDevice"));
    SR_TRY(hip_status(hipSetDevice(device), "hipSetDevice"));
    void* p = nullptr;
    float* scratch = nullptr;
    hipError_t e = hipMalloc(&p, 4 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(p, 0, 4 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    // the address of this device's copy of the scratch array, with the device current
    if (e == hipSuccess) e = sr::scratch_address(device, &scratch);
    hipSetDevice(prev);
    if (e != hipSuccess) {
        if (p) hipFree(p);
        return hip_status(e, "sr_create");
    }
    sr_ctx* c = new (std::nothrow) sr_ctx{device, (uint32_t*)p, scratch};
    if (!c) {
        hipFree(p);
        return fail(SR_ERR_ARG, "out of host memory");
    }
    *ctx_out_host = c;
    return SR_OK;
}

sr_status sr_destroy(sr_ctx* ctx) {
    if (!ctx) return SR_OK;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    const hipError_t e = hipFree(ctx->status);
    hipSetDevice(prev);
    delete ctx;
    return hip_status(e, "sr_destroy");
}

sr_status sr_read_status(sr_ctx* ctx, void* stream, int32_t clear, uint32_t* status_bits_host,
                         uint64_t* needed_capacity_host) {
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    uint32_t w[4] = {0, 0, 0, 0};
    SR_TRY(hip_status(hipStreamSynchronize(s), "sr_read_status: stream"));
    SR_TRY(hip_status(hipMemcpy(w, ctx->status, sizeof(w), hipMemcpyDeviceToHost), "sr_read_status: copy"));
    if (clear) {
        SR_TRY(hip_status(sr::fill_u32(ctx->status, 0u, 4, s), "sr_read_status: clear"));
        SR_TRY(hip_status(hipStreamSynchronize(s), "sr_read_status: clear"));
    }
    if (status_bits_host) *status_bits_host = w[0];
    if (needed_capacity_host) *needed_capacity_host = w[1];
    if (w[0] & SR_STATUS_CAPACITY)
        return fail(SR_ERR_CAPACITY, "instance capacity exceeded: %u instances needed", w[1]);
    return SR_OK;
}

sr_status sr_clear_status(sr_ctx* ctx, void* stream) {
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::fill_u32(ctx->status, 0u, 4, (hipStream_t)stream), "sr_clear_status");
}

int32_t sr_tile_supported(int32_t tile_w, int32_t tile_h) { return sr::tile_shape_supported(tile_w, tile_h) ? 1 : 0; }

int32_t sr_bwd_batch_supported(int32_t tile_w, int32_t tile_h, int32_t batch) {
    return sr::bwd_batch_supported(tile_w, tile_h, batch) ? 1 : 0;
}

sr_status sr_layout_views(sr_camera* cams_host, int32_t V, int32_t tile_w, int32_t tile_h,
                          int64_t* total_pixels_host, int32_t* total_tiles_host) {
    if (V < 0) return fail(SR_ERR_ARG, "V = %d < 0", V);
    if (tile_w < 1 || tile_h < 1) return fail(SR_ERR_ARG, "tile shape %dx%d", tile_w, tile_h);
    if (V > 0 && !cams_host) return fail(SR_ERR_ARG, "cams_host is NULL");
    int64_t pix = 0, tiles = 0, groups = 0;
    for (int v = 0; v < V; ++v) {
        sr_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
            return fail(SR_ERR_ARG, "view %d: size %dx%d outside [1, 65535]", v, c.width, c.height);
        c.tiles_x = (c.width + tile_w - 1) / tile_w;
        c.tiles_y = (c.height + tile_h - 1) / tile_h;
        c.tile_offset = (int32_t)tiles;
        c.pix_offset = pix;
        c.groups_x = (c.tiles_x + SR_TILE_GROUP - 1) / SR_TILE_GROUP;
        c.group_offset = (int32_t)groups;
        groups += (int64_t)c.groups_x * ((c.tiles_y + SR_TILE_GROUP - 1) / SR_TILE_GROUP);
        tiles += (int64_t)c.tiles_x * c.tiles_y;
        pix += (int64_t)c.width * c.height;
        if (tiles > 0x7FFFFFFF) return fail(SR_ERR_ARG, "too many tiles");
    }
    if (total_pixels_host) *total_pixels_host = pix;
    if (total_tiles_host) *total_tiles_host = (int32_t)tiles;
    return SR_OK;
}

sr_status sr_preprocess(sr_ctx* ctx, const sr_config* cfg, int32_t N, const float* means, const float* scales,
                        const float* quats, const float* opac, const float* sh, int32_t V,
                        const sr_camera* cams_host, const sr_camera* cams_dev, float* geom, float* app,
                        uint16_t* rect, uint32_t* tiles_touched, uint32_t* depth_key, uint8_t* in_frustum,
                        void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, nullptr, nullptr));
    if (N > 0) {
        SR_NEED(means); SR_NEED(scales); SR_NEED(quats); SR_NEED(opac);
        if (app) SR_NEED(sh);
        if (V > 0) { SR_NEED(geom); SR_NEED(rect); SR_NEED(tiles_touched); SR_NEED(depth_key); }
    }
    if (N == 0) return SR_OK;                      // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_preprocess(*cfg, N, means, scales, quats, opac, sh, V, cams_dev, geom, app, rect,
                                            tiles_touched, depth_key, in_frustum, (hipStream_t)stream),
                      "sr_preprocess");
}

sr_status sr_bin_workspace_size(int32_t N, int32_t V, uint32_t inst_capacity, size_t* bytes_host) {
    SR_TRY(check_nv(N, V));
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    SR_NEED(bytes_host);
    *bytes_host = sr::bin_workspace_bytes((uint64_t)N * (uint64_t)V, inst_capacity);
    return SR_OK;
}

sr_status sr_bin_and_sort(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                          const sr_camera* cams_dev, const uint16_t* rect, const uint32_t* tiles_touched,
                          const uint32_t* depth_key, void* workspace, size_t ws_bytes, uint32_t inst_capacity,
                          uint32_t* vals, uint64_t* keys64, uint32_t* ranges, uint32_t* counters, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    if (N >= (1 << SR_INST_ID_BITS))
        return fail(SR_ERR_UNSUPPORTED, "N = %d: binned surfel ids hold %d bits", N, SR_INST_ID_BITS);
    int total_tiles = 0, total_groups = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr,
                       &total_groups));
    SR_NEED(counters);
    if (total_tiles > 0) SR_NEED(ranges);
    const size_t need = sr::bin_workspace_bytes((uint64_t)N * (uint64_t)V, inst_capacity);
    if (ws_bytes < need) return fail(SR_ERR_ARG, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((uint64_t)N * V > 0) {
        SR_NEED(workspace); SR_NEED(rect); SR_NEED(tiles_touched); SR_NEED(depth_key);
        if (inst_capacity > 0) SR_NEED(vals);
    }
    if (inst_capacity == 0xFFFFFFFFu) return fail(SR_ERR_ARG, "inst_capacity must be below 2^32 - 1");
    SR_TRY(check_ctx(ctx));
    const bool count_only = inst_capacity == 0 && vals == nullptr;
    return hip_status(sr::launch_bin_and_sort(*cfg, N, V, total_tiles, total_groups, cams_dev, rect, tiles_touched,
                                              depth_key, workspace, inst_capacity, vals, keys64, ranges, counters,
                                              ctx->status, count_only, (hipStream_t)stream),
                      "sr_bin_and_sort");
}

namespace {

// Statistics arguments of the forward and the training step: none, hits
// alone (the usage count), or hits with both maxima.
sr_status check_stats(const uint32_t* hits, const float* max_alpha, const float* max_weight) {
    if ((max_alpha == nullptr) != (max_weight == nullptr))
        return fail(SR_ERR_ARG, "max_alpha and max_weight must be given together");
    if (max_alpha && !hits) return fail(SR_ERR_ARG, "max_alpha and max_weight need hits");
    return SR_OK;
}

sr_status clear_stats(int32_t N, uint32_t* hits, float* max_alpha, float* max_weight, hipStream_t s) {
    if (N == 0) return SR_OK;
    if (hits) SR_TRY(hip_status(sr::fill_f32((float*)hits, 0.f, (uint64_t)N, s), "clear hits"));
    if (max_alpha) SR_TRY(hip_status(sr::fill_f32(max_alpha, 0.f, (uint64_t)N, s), "clear max_alpha"));
    if (max_weight) SR_TRY(hip_status(sr::fill_f32(max_weight, 0.f, (uint64_t)N, s), "clear max_weight"));
    return SR_OK;
}

}  // namespace

sr_status sr_render_forward(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                            const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                            const uint32_t* ranges, float* color, float* alpha, float* depth, float* normal,
                            float* dist, float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha,
                            float* max_weight, float* median_depth, uint32_t* median_contrib,
                            const uint32_t* tile_order, uint32_t* tile_cost, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (total_tiles > 0) {
        SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges);
        SR_NEED(color); SR_NEED(alpha); SR_NEED(depth); SR_NEED(normal); SR_NEED(dist); SR_NEED(T_final);
        SR_NEED(n_contrib);
    }
    SR_TRY(check_stats(hits, max_alpha, max_weight));
    if ((median_depth == nullptr) != (median_contrib == nullptr))
        return fail(SR_ERR_ARG, "median_depth and median_contrib must be given together");
    if (N == 0 && total_tiles == 0) return SR_OK;  // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE)) SR_TRY(clear_stats(N, hits, max_alpha, max_weight, s));
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, app, nullptr, vals, ranges,
                                            color, alpha, depth, normal, dist, T_final, n_contrib, hits, max_alpha,
                                            max_weight, nullptr, median_depth, median_contrib, tile_order,
                                            tile_cost, ctx->status, s),
                      "sr_render_forward");
}

namespace {

sr_status check_backward_raster(const sr_config* cfg, int N, int V, const sr_camera* cams_host,
                                const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                                const uint32_t* ranges, const float* alpha, const float* depth, const float* dist,
                                const float* T_final, const uint32_t* n_contrib, const float* grad_rec,
                                int* total_tiles) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, total_tiles, nullptr));
    if (N > 0 && V > 0) {
        SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges);
        SR_NEED(alpha); SR_NEED(depth); SR_NEED(dist); SR_NEED(T_final); SR_NEED(n_contrib); SR_NEED(grad_rec);
    }
    return SR_OK;
}

sr_status check_backward_project(const sr_config* cfg, int N, int V, const sr_camera* cams_host,
                                 const sr_camera* cams_dev, const float* means, const float* scales,
                                 const float* quats, const float* sh, const float* geom, const float* app,
                                 const float* grad_rec, const float* g_means, const float* g_scales,
                                 const float* g_quats, const float* g_opac, const float* g_sh) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, nullptr, nullptr));
    if (N > 0 && V > 0) {
        SR_NEED(means); SR_NEED(scales); SR_NEED(quats); SR_NEED(sh); SR_NEED(geom); SR_NEED(app);
        SR_NEED(grad_rec); SR_NEED(g_means); SR_NEED(g_scales); SR_NEED(g_quats); SR_NEED(g_opac); SR_NEED(g_sh);
    }
    return SR_OK;
}

}  // namespace

sr_status sr_backward_raster(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                             const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                             const uint32_t* ranges, const float* alpha, const float* depth, const float* dist,
                             const float* T_final, const uint32_t* n_contrib, const float* dL_dcolor,
                             const float* dL_dalpha, const float* dL_ddepth, const float* dL_dnormal,
                             const float* dL_ddist, const uint32_t* median_contrib, const float* dL_dmedian,
                             float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order, void* stream) {
    int total_tiles = 0;
    SR_TRY(check_backward_raster(cfg, N, V, cams_host, cams_dev, geom, app, vals, ranges, alpha, depth, dist, T_final,
                                 n_contrib, grad_rec, &total_tiles));
    if (dL_dmedian && !median_contrib) return fail(SR_ERR_ARG, "dL_dmedian needs median_contrib");
    if (N == 0 || V == 0) return SR_OK;
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_render_bwd(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, alpha, depth,
                                            dist, T_final, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dnormal,
                                            dL_ddist, median_contrib, dL_dmedian, grad_rec, grad_marks, tile_order,
                                            ctx->status, (hipStream_t)stream),
                      "sr_backward_raster");
}

sr_status sr_backward_project(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                              const sr_camera* cams_dev, const float* means, const float* scales, const float* quats,
                              const float* sh, const float* geom, const float* app, uint32_t* tiles_touched,
                              float* grad_rec, float* g_means, float* g_scales, float* g_quats, float* g_opac,
                              float* g_sh, float* densify_grad, uint32_t* densify_count, void* stream) {
    SR_TRY(check_backward_project(cfg, N, V, cams_host, cams_dev, means, scales, quats, sh, geom, app, grad_rec,
                                  g_means, g_scales, g_quats, g_opac, g_sh));
    if ((densify_grad || densify_count) && !tiles_touched)
        return fail(SR_ERR_ARG, "the density statistics need tiles_touched (the views each surfel is seen in)");
    if ((cfg->flags & SR_FLAG_MARKED_GRADIENTS) && !tiles_touched)
        return fail(SR_ERR_ARG, "SR_FLAG_MARKED_GRADIENTS needs tiles_touched (the marks live there)");
    if (N == 0 || V == 0) return SR_OK;
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_preprocess_bwd(*cfg, N, means, scales, quats, sh, V, cams_dev, geom, app,
                                                tiles_touched, grad_rec, g_means, g_scales, g_quats, g_opac, g_sh,
                                                densify_grad, densify_count, (hipStream_t)stream),
                      "sr_backward_project");
}

sr_status sr_render_backward(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                             const sr_camera* cams_dev, const float* means, const float* scales, const float* quats,
                             const float* opac, const float* sh, const float* geom, const float* app,
                             const uint32_t* vals, const uint32_t* ranges, const float* alpha, const float* depth,
                             const float* dist, const float* T_final, const uint32_t* n_contrib,
                             const float* dL_dcolor, const float* dL_dalpha, const float* dL_ddepth,
                             const float* dL_dnormal, const float* dL_ddist, const uint32_t* median_contrib,
                             const float* dL_dmedian, float* grad_rec, float* g_means, float* g_scales,
                             float* g_quats, float* g_opac, float* g_sh, void* stream) {
    int total_tiles = 0;
    (void)opac;
    SR_TRY(check_backward_raster(cfg, N, V, cams_host, cams_dev, geom, app, vals, ranges, alpha, depth, dist, T_final,
                                 n_contrib, grad_rec, &total_tiles));
    if (dL_dmedian && !median_contrib) return fail(SR_ERR_ARG, "dL_dmedian needs median_contrib");
    SR_TRY(check_backward_project(cfg, N, V, cams_host, cams_dev, means, scales, quats, sh, geom, app, grad_rec,
                                  g_means, g_scales, g_quats, g_opac, g_sh));
    if (N == 0 || V == 0) return SR_OK;
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    SR_TRY(hip_status(sr::fill_f32(grad_rec, 0.f, (uint64_t)V * N * SR_GRAD_STRIDE, s), "clear grad_rec"));
    SR_TRY(hip_status(sr::launch_render_bwd(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, alpha, depth,
                                            dist, T_final, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dnormal,
                                            dL_ddist, median_contrib, dL_dmedian, grad_rec, nullptr, nullptr,
                                            ctx->status, s),
                      "render backward"));
    sr_config pcfg = *cfg;
    pcfg.flags &= ~SR_FLAG_MARKED_GRADIENTS;     // no marks here: every record is read
    return hip_status(sr::launch_preprocess_bwd(pcfg, N, means, scales, quats, sh, V, cams_dev, geom, app, nullptr,
                                                grad_rec, g_means, g_scales, g_quats, g_opac, g_sh, nullptr,
                                                nullptr, s),
                      "projection backward");
}

sr_status sr_loss_workspace_size(int32_t V, const sr_camera* cams_host, size_t* bytes_host) {
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    SR_NEED(bytes_host);
    if (V > 0) SR_NEED(cams_host);
    int64_t mhw = 0;
    int mt = 0;
    for (int v = 0; v < V; ++v) {
        if (cams_host[v].width < 0 || cams_host[v].height < 0) return fail(SR_ERR_ARG, "view %d: negative size", v);
        const int64_t hw = (int64_t)cams_host[v].width * cams_host[v].height;
        if (hw > mhw) mhw = hw;
        const int t = sr::reg_tile_count(cams_host[v].width, cams_host[v].height);
        if (t > mt) mt = t;
    }
    *bytes_host = sr::loss_workspace_bytes(V, mhw, mt);
    return SR_OK;
}

sr_status sr_background_loss(sr_ctx* ctx, int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* alpha,
                             const uint8_t* mask, const float* color, const float* target, float gamma, float w_c,
                             void* workspace, size_t ws_bytes, float* loss, float* dL_dalpha, float* dL_dcolor,
                             void* stream) {
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    if (V == 0) return SR_OK;
    SR_NEED(cams_host); SR_NEED(cams_dev); SR_NEED(alpha); SR_NEED(mask); SR_NEED(loss); SR_NEED(workspace);
    if ((color == nullptr) != (target == nullptr)) return fail(SR_ERR_ARG, "color and target go together");
    if (dL_dcolor && !color) return fail(SR_ERR_ARG, "dL_dcolor needs color and target");
    int64_t mhw = 0, pix = 0;
    for (int v = 0; v < V; ++v) {
        const sr_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1) return fail(SR_ERR_ARG, "view %d: empty", v);
        if (c.pix_offset != pix) return fail(SR_ERR_ARG, "view %d: pix_offset not laid out", v);
        pix += (int64_t)c.width * c.height;
        if ((int64_t)c.width * c.height > mhw) mhw = (int64_t)c.width * c.height;
    }
    if (ws_bytes < sr::loss_workspace_bytes(V, mhw, 0)) return fail(SR_ERR_ARG, "loss workspace too small");
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_loss(V, mhw, cams_dev, alpha, mask, color, target, gamma, w_c, workspace, loss,
                                      dL_dalpha, dL_dcolor, (hipStream_t)stream),
                      "sr_background_loss");
}

sr_status sr_regularizer_loss(sr_ctx* ctx, int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* alpha,
                              const float* depth, const float* normal, const float* dist, const float* median,
                              float w_dist, float w_normal, void* workspace, size_t ws_bytes, float* loss,
                              float* dL_dalpha, float* dL_ddepth, float* dL_dnormal, float* dL_ddist,
                              float* dL_dmedian, void* stream) {
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    if (V == 0) return SR_OK;
    SR_NEED(cams_host); SR_NEED(cams_dev); SR_NEED(alpha); SR_NEED(depth); SR_NEED(normal); SR_NEED(dist);
    SR_NEED(loss); SR_NEED(workspace); SR_NEED(dL_dalpha); SR_NEED(dL_ddepth); SR_NEED(dL_dnormal);
    SR_NEED(dL_ddist);
    if ((median == nullptr) != (dL_dmedian == nullptr)) return fail(SR_ERR_ARG, "median and dL_dmedian go together");
    int64_t pix = 0, tt = 0;
    int mt = 0;
    for (int v = 0; v < V; ++v) {
        const sr_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1) return fail(SR_ERR_ARG, "view %d: empty", v);
        if (c.pix_offset != pix) return fail(SR_ERR_ARG, "view %d: pix_offset not laid out", v);
        if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(SR_ERR_ARG, "view %d: focal lengths must be positive", v);
        pix += (int64_t)c.width * c.height;
        const int t = sr::reg_tile_count(c.width, c.height);
        if (t > mt) mt = t;
        tt += t;
    }
    if (tt > 0x7FFFFFFF) return fail(SR_ERR_ARG, "too many regulariser tiles");
    if (ws_bytes < sr::loss_workspace_bytes(V, 0, mt)) return fail(SR_ERR_ARG, "regularizer workspace too small");
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_reg_loss(V, mt, (int)tt, cams_dev, alpha, depth, normal, dist, median, w_dist, w_normal,
                                          workspace, loss, dL_dalpha, dL_ddepth, dL_dnormal, dL_ddist, dL_dmedian,
                                          (hipStream_t)stream),
                      "sr_regularizer_loss");
}

static sr_status ssim_sizes(int32_t V, const sr_camera* cams_host, int* max_slots, int64_t* P,
                            int* total_slots = nullptr) {
    int64_t pix = 0, tot = 0;
    int ms = 0;
    for (int v = 0; v < V; ++v) {
        const sr_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1) return fail(SR_ERR_ARG, "view %d: empty", v);
        if (c.pix_offset != pix) return fail(SR_ERR_ARG, "view %d: pix_offset not laid out", v);
        pix += (int64_t)c.width * c.height;
        const int t = sr::ssim_slots(c.width, c.height);
        if (t > ms) ms = t;
        tot += t;
    }
    if (tot > 0x7FFFFFFF) return fail(SR_ERR_ARG, "too many SSIM tiles");
    *max_slots = ms;
    *P = pix;
    if (total_slots) *total_slots = (int)tot;
    return SR_OK;
}

sr_status sr_ssim_workspace_size(int32_t V, const sr_camera* cams_host, int32_t with_grad, size_t* bytes_host) {
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    SR_NEED(bytes_host);
    if (V == 0) { *bytes_host = 0; return SR_OK; }
    SR_NEED(cams_host);
    int ms = 0;
    int64_t P = 0;
    SR_TRY(ssim_sizes(V, cams_host, &ms, &P));
    *bytes_host = sr::ssim_workspace_bytes(V, ms, P, with_grad != 0);
    return SR_OK;
}

sr_status sr_ssim_loss(sr_ctx* ctx, int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* color,
                       const float* target, const uint8_t* mask, float w_s, void* workspace, size_t ws_bytes,
                       float* out, float* dL_dcolor, void* stream) {
    if (V < 0) return fail(SR_ERR_ARG, "V < 0");
    if (V == 0) return SR_OK;
    SR_NEED(cams_host); SR_NEED(cams_dev); SR_NEED(color); SR_NEED(target); SR_NEED(mask); SR_NEED(workspace);
    SR_NEED(out);
    int ms = 0, tot = 0;
    int64_t P = 0;
    SR_TRY(ssim_sizes(V, cams_host, &ms, &P, &tot));
    if (ws_bytes < sr::ssim_workspace_bytes(V, ms, P, dL_dcolor != nullptr))
        return fail(SR_ERR_ARG, "ssim workspace too small");
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_ssim(V, ms, tot, P, cams_dev, color, target, mask, w_s, workspace, out, dL_dcolor,
                                      (hipStream_t)stream),
                      "sr_ssim_loss");
}

sr_status sr_preprocess_3d(sr_ctx* ctx, const sr_config* cfg, int32_t N, const float* means, const float* scales,
                           const float* quats, const float* opac, int32_t V, const sr_camera* cams_host,
                           const sr_camera* cams_dev, float* geom3, uint16_t* rect, uint32_t* tiles_touched,
                           uint32_t* depth_key, uint8_t* in_frustum, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, nullptr, nullptr));
    if (N > 0) {
        SR_NEED(means); SR_NEED(scales); SR_NEED(quats); SR_NEED(opac);
        if (V > 0) { SR_NEED(geom3); SR_NEED(rect); SR_NEED(tiles_touched); SR_NEED(depth_key); }
    }
    if (N == 0) return SR_OK;                      // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_preprocess3d(*cfg, N, means, scales, quats, opac, V, cams_dev, geom3, rect,
                                              tiles_touched, depth_key, in_frustum, (hipStream_t)stream),
                      "sr_preprocess_3d");
}

sr_status sr_prune_stats_3d(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                              const sr_camera* cams_dev, const float* geom3, const uint32_t* vals,
                              const uint32_t* ranges, uint32_t* hits, float* max_alpha, float* max_weight,
                              void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (N > 0) { SR_NEED(hits); SR_NEED(max_alpha); SR_NEED(max_weight); }
    if (total_tiles > 0) { SR_NEED(geom3); SR_NEED(vals); SR_NEED(ranges); }
    if (N == 0 && total_tiles == 0) return SR_OK;  // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE) && N > 0) {
        SR_TRY(hip_status(sr::fill_f32((float*)hits, 0.f, (uint64_t)N, s), "clear hits"));
        SR_TRY(hip_status(sr::fill_f32(max_alpha, 0.f, (uint64_t)N, s), "clear max_alpha"));
        SR_TRY(hip_status(sr::fill_f32(max_weight, 0.f, (uint64_t)N, s), "clear max_weight"));
    }
    return hip_status(sr::launch_prune3d(*cfg, N, V, total_tiles, cams_dev, geom3, vals, ranges, hits, max_alpha,
                                         max_weight, ctx->status, s),
                      "sr_prune_stats_3d");
}

sr_status sr_compact_workspace_size(int32_t N, size_t* bytes_host) {
    if (N < 0) return fail(SR_ERR_ARG, "N < 0");
    SR_NEED(bytes_host);
    *bytes_host = sr::compact_workspace_bytes(N);
    return SR_OK;
}

sr_status sr_compact_surfels(sr_ctx* ctx, int32_t N, const uint8_t* prune_mask, const float* opac, float min_opacity,
                             int32_t n_arrays, const float* const* src_host, float* const* dst_host,
                             const int32_t* widths_host, void* workspace, size_t ws_bytes, uint32_t* n_kept,
                             void* stream) {
    if (N < 0) return fail(SR_ERR_ARG, "N < 0");
    if (n_arrays < 0 || n_arrays > SR_COMPACT_MAX_ARRAYS)
        return fail(SR_ERR_ARG, "n_arrays must be in [0, %d]", SR_COMPACT_MAX_ARRAYS);
    SR_NEED(n_kept); SR_NEED(workspace);
    if (N > 0) SR_NEED(prune_mask);
    if (n_arrays > 0) { SR_NEED(src_host); SR_NEED(dst_host); SR_NEED(widths_host); }
    for (int a = 0; a < n_arrays; ++a) {
        if (widths_host[a] < 1) return fail(SR_ERR_ARG, "array %d: width must be positive", a);
        if (N > 0 && (!src_host[a] || !dst_host[a])) return fail(SR_ERR_ARG, "array %d: missing pointer", a);
        if (N > 0 && (const void*)src_host[a] == (const void*)dst_host[a])
            return fail(SR_ERR_ARG, "array %d: dst aliases src", a);
    }
    if (ws_bytes < sr::compact_workspace_bytes(N)) return fail(SR_ERR_ARG, "compaction workspace too small");
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_compact(N, prune_mask, opac, min_opacity, n_arrays, src_host, dst_host,
                                         (const int*)widths_host, workspace, n_kept, (hipStream_t)stream),
                      "sr_compact_surfels");
}

sr_status sr_prune_stats(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                           const sr_camera* cams_dev, const float* geom, const uint16_t* rect, const uint32_t* vals,
                           const uint32_t* ranges, uint32_t* hits, float* max_alpha, float* max_weight,
                           void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (N > 0) { SR_NEED(hits); SR_NEED(max_alpha); SR_NEED(max_weight); }
    if (total_tiles > 0) { SR_NEED(geom); SR_NEED(vals); SR_NEED(ranges); }
    if (N == 0 && total_tiles == 0) return SR_OK;  // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE) && N > 0) {
        SR_TRY(hip_status(sr::fill_f32((float*)hits, 0.f, (uint64_t)N, s), "clear hits"));
        SR_TRY(hip_status(sr::fill_f32(max_alpha, 0.f, (uint64_t)N, s), "clear max_alpha"));
        SR_TRY(hip_status(sr::fill_f32(max_weight, 0.f, (uint64_t)N, s), "clear max_weight"));
    }
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, nullptr, rect, vals, ranges,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, hits,
                                            max_alpha, max_weight, nullptr, nullptr, nullptr, nullptr, nullptr,
                                            ctx->status, s),
                      "sr_prune_stats");
}

namespace {

// The fused training step with its per-tile loss partials in tile_loss
// (the caller's buffer, or the context's scratch array).
sr_status train_step(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                     const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                     const uint32_t* ranges, const uint8_t* mask, const float* target, float gamma, float w_c,
                     float* color, float* alpha, float* depth, float* normal, float* dist, float* T_final,
                     uint32_t* n_contrib, uint32_t* hits, float* max_alpha, float* max_weight, float* tile_loss,
                     float* loss, float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order,
                     uint32_t* tile_cost, void* stream, bool noalloc) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (noalloc && total_tiles > SR_NOALLOC_MAX_TILES)
        return fail(SR_ERR_ARG, "%d tiles exceed the scratch array's %d (SR_NOALLOC_MAX_TILES)", total_tiles,
                    SR_NOALLOC_MAX_TILES);
    if (total_tiles > 0) {
        SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges); SR_NEED(mask); SR_NEED(target);
        SR_NEED(color); SR_NEED(alpha); SR_NEED(depth); SR_NEED(normal); SR_NEED(dist); SR_NEED(T_final);
        SR_NEED(n_contrib); SR_NEED(loss); SR_NEED(grad_rec);
        if (!noalloc) SR_NEED(tile_loss);
    }
    SR_TRY(check_stats(hits, max_alpha, max_weight));
    if (N == 0 && total_tiles == 0) return SR_OK;  // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    if (noalloc) {
        if (!ctx->scratch) return fail(SR_ERR_STATE, "the context has no scratch array address");
        tile_loss = ctx->scratch;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE)) SR_TRY(clear_stats(N, hits, max_alpha, max_weight, s));
    if (total_tiles == 0) return SR_OK;
    SR_TRY(hip_status(sr::launch_train_raster(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, mask, target,
                                              gamma, w_c, color, alpha, depth, normal, dist, T_final, n_contrib, hits,
                                              max_alpha, max_weight, tile_loss, grad_rec, grad_marks, tile_order,
                                              tile_cost, ctx->status, s),
                      "sr_train_step_raster"));
    return hip_status(sr::launch_loss_from_tiles(V, cams_dev, tile_loss, gamma, w_c, loss, s), "loss totals");
}

}  // namespace

sr_status sr_train_step_raster(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                               const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                               const uint32_t* ranges, const uint8_t* mask, const float* target, float gamma,
                               float w_c, float* color, float* alpha, float* depth, float* normal, float* dist,
                               float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha,
                               float* max_weight, float* tile_loss, float* loss, float* grad_rec,
                               uint32_t* grad_marks, const uint32_t* tile_order, uint32_t* tile_cost, void* stream) {
    return train_step(ctx, cfg, N, V, cams_host, cams_dev, geom, app, vals, ranges, mask, target, gamma, w_c, color,
                      alpha, depth, normal, dist, T_final, n_contrib, hits, max_alpha, max_weight, tile_loss, loss,
                      grad_rec, grad_marks, tile_order, tile_cost, stream, false);
}

sr_status sr_train_step_raster_noalloc(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V,
                                       const sr_camera* cams_host, const sr_camera* cams_dev, const float* geom,
                                       const float* app, const uint32_t* vals, const uint32_t* ranges,
                                       const uint8_t* mask, const float* target, float gamma, float w_c,
                                       float* color, float* alpha, float* depth, float* normal, float* dist,
                                       float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha,
                                       float* max_weight, float* loss, float* grad_rec, uint32_t* grad_marks,
                                       const uint32_t* tile_order, uint32_t* tile_cost, void* stream) {
    return train_step(ctx, cfg, N, V, cams_host, cams_dev, geom, app, vals, ranges, mask, target, gamma, w_c, color,
                      alpha, depth, normal, dist, T_final, n_contrib, hits, max_alpha, max_weight, nullptr, loss,
                      grad_rec, grad_marks, tile_order, tile_cost, stream, true);
}

sr_status sr_render_count(sr_ctx* ctx, const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                          const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                          const uint32_t* ranges, uint64_t* counts, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    SR_NEED(counts);
    if (total_tiles > 0) { SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges); }
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    SR_TRY(hip_status(sr::fill_f32((float*)counts, 0.f, 10, s), "clear counts"));
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, app, nullptr, vals, ranges,
                                            nullptr,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                            nullptr, (unsigned long long*)counts, nullptr, nullptr, nullptr, nullptr,
                                            ctx->status, s),
                      "sr_render_count");
}

sr_status sr_prune_mask(sr_ctx* ctx, int32_t N, const float* max_alpha, float tau, uint8_t* prune_mask,
                        void* stream) {
    if (N < 0) return fail(SR_ERR_ARG, "N < 0");
    if (N > 0) { SR_NEED(max_alpha); SR_NEED(prune_mask); }
    if (N == 0) return SR_OK;                      // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_prune_mask(N, max_alpha, tau, ctx->status, prune_mask, (hipStream_t)stream),
                      "sr_prune_mask");
}

sr_status sr_tile_order_workspace_size(int32_t T, size_t* bytes_host) {
    if (T < 0) return fail(SR_ERR_ARG, "T = %d < 0", T);
    SR_NEED(bytes_host);
    *bytes_host = T > 0 ? sr::tile_order_workspace(T) : 0;
    return SR_OK;
}

sr_status sr_tile_order(sr_ctx* ctx, int32_t T, const uint32_t* tile_cost, void* workspace, size_t ws_bytes,
                        uint32_t* tile_order, void* stream) {
    if (T < 0) return fail(SR_ERR_ARG, "T = %d < 0", T);
    if (T == 0) return SR_OK;
    SR_NEED(tile_cost); SR_NEED(workspace); SR_NEED(tile_order);
    if (ws_bytes < sr::tile_order_workspace(T))
        return fail(SR_ERR_ARG, "workspace of %zu bytes < %zu", ws_bytes, sr::tile_order_workspace(T));
    SR_TRY(check_ctx(ctx));
    return hip_status(sr::launch_tile_order(T, tile_cost, workspace, tile_order, (hipStream_t)stream),
                      "sr_tile_order");
}

sr_status sr_workspace_size(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                            uint32_t inst_capacity, size_t* bytes_host) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    SR_NEED(bytes_host);
    if (V > 0) SR_NEED(cams_host);
    int total_tiles = 0;
    // the layout is checked against itself (cams_dev is not needed here)
    SR_TRY(check_views(cams_host, cams_host, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    size_t b = sr::bin_workspace_bytes((uint64_t)N * (uint64_t)V, inst_capacity);
    size_t x = 0;
    SR_TRY(sr_loss_workspace_size(V, cams_host, &x));
    b = std::max(b, x);
    SR_TRY(sr_ssim_workspace_size(V, cams_host, 1, &x));
    b = std::max(b, x);
    b = std::max(b, total_tiles > 0 ? sr::tile_order_workspace(total_tiles) : (size_t)0);
    b = std::max(b, sr::compact_workspace_bytes(N));
    *bytes_host = b;
    return SR_OK;
}

namespace {

// ---- the whole pruning pass ---------------------------------------------------

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Chunk k covers views [k*vpc, min(V, (k+1)*vpc)).
struct PruneLayout {
    int chunks = 0, max_views = 0, max_tiles = 0;
    size_t cams = 0, geom = 0, rect = 0, tt = 0, dk = 0, ranges = 0, vals = 0, counters = 0, bin = 0, bytes = 0;
};

sr_status prune_layout(const sr_config* cfg, int prim, int N, int V, const sr_camera* cams_host, int vpc,
                       uint32_t cap, PruneLayout* L) {
    if (prim != SR_PRIM_SURFEL && prim != SR_PRIM_GAUSS3D) return fail(SR_ERR_ARG, "prim %d is not a primitive", prim);
    if (vpc < 1) return fail(SR_ERR_ARG, "views_per_chunk = %d < 1", vpc);
    SR_TRY(check_nv(N, std::min(V, vpc)));
    if (N >= (1 << SR_INST_ID_BITS))
        return fail(SR_ERR_UNSUPPORTED, "N = %d: binned surfel ids hold %d bits", N, SR_INST_ID_BITS);
    if (cap == 0xFFFFFFFFu) return fail(SR_ERR_ARG, "inst_capacity must be below 2^32 - 1");
    L->chunks = (V + vpc - 1) / vpc;
    L->max_views = std::min(V, vpc);
    for (int k = 0; k < L->chunks; ++k) {
        const int v0 = k * vpc, v1 = std::min(V, v0 + vpc);
        const int64_t t = (v1 < V ? (int64_t)cams_host[v1].tile_offset
                                  : (int64_t)cams_host[V - 1].tile_offset +
                                        (int64_t)cams_host[V - 1].tiles_x * cams_host[V - 1].tiles_y) -
                          cams_host[v0].tile_offset;
        L->max_tiles = std::max(L->max_tiles, (int)t);
    }
    const uint64_t VN = (uint64_t)L->max_views * (uint64_t)N;
    const int gstride = prim == SR_PRIM_SURFEL ? SR_GEOM_STRIDE : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L->cams = take((size_t)L->max_views * sizeof(sr_camera));
    L->geom = take(VN * gstride * sizeof(float));
    L->rect = take(VN * 4 * sizeof(uint16_t));
    L->tt = take(VN * sizeof(uint32_t));
    L->dk = take(VN * sizeof(uint32_t));
    L->ranges = take((size_t)2 * L->max_tiles * sizeof(uint32_t));
    L->vals = take((size_t)cap * sizeof(uint32_t));
    L->counters = take((size_t)SR_COUNTERS * sizeof(uint32_t) * L->chunks);
    L->bin = take(sr::bin_workspace_bytes(VN, cap));
    L->bytes = off;
    return SR_OK;
}

// One chunk's cameras as a batch of their own: host copy (validation and
// launch geometry) and device copy (rebased by a kernel, no host copy).
void chunk_cams(const sr_camera* cams_host, int v0, int v1, std::vector<sr_camera>& hc) {
    hc.assign(cams_host + v0, cams_host + v1);
    for (auto& c : hc) {
        c.tile_offset -= cams_host[v0].tile_offset;
        c.pix_offset -= cams_host[v0].pix_offset;
        c.group_offset -= cams_host[v0].group_offset;
    }
}

// Projection (no shading) and binning of views [v0, v1) into the workspace;
// count_only: instance count only (capacity planning).
sr_status prune_chunk_bin(sr_ctx* ctx, const sr_config& cfg, int prim, int N, const float* means,
                          const float* scales, const float* quats, const float* opac, const sr_camera* cams_host,
                          const sr_camera* cams_dev, int v0, int v1, uint8_t* in_frustum, bool or_frustum,
                          char* ws, const PruneLayout& L, uint32_t cap, bool count_only, int chunk, hipStream_t s,
                          std::vector<sr_camera>& hc, int* tiles_out) {
    chunk_cams(cams_host, v0, v1, hc);
    const int Vc = v1 - v0;
    int tiles = 0, groups = 0;
    SR_TRY(check_views(hc.data(), hc.data(), Vc, cfg.tile_w, cfg.tile_h, nullptr, &tiles, nullptr, &groups));
    sr_camera* dc = (sr_camera*)(ws + L.cams);
    SR_TRY(hip_status(sr::launch_rebase_cams(cams_dev + v0, Vc, dc, s), "prune pass: cameras"));
    float* geom = (float*)(ws + L.geom);
    uint16_t* rect = (uint16_t*)(ws + L.rect);
    uint32_t* tt = (uint32_t*)(ws + L.tt);
    uint32_t* dk = (uint32_t*)(ws + L.dk);
    sr_config c = cfg;
    // in_frustum: cleared by the first chunk unless accumulating, then OR
    c.flags = or_frustum ? (c.flags | SR_FLAG_ACCUMULATE) : (c.flags & ~SR_FLAG_ACCUMULATE);
    if (prim == SR_PRIM_SURFEL)
        SR_TRY(hip_status(sr::launch_preprocess(c, N, means, scales, quats, opac, nullptr, Vc, dc, geom, nullptr, rect,
                                                tt, dk, in_frustum, s),
                          "prune pass: projection"));
    else
        SR_TRY(hip_status(sr::launch_preprocess3d(c, N, means, scales, quats, opac, Vc, dc, geom, rect, tt, dk,
                                                  in_frustum, s),
                          "prune pass: projection"));
    uint32_t* counters = (uint32_t*)(ws + L.counters) + (size_t)SR_COUNTERS * chunk;
    SR_TRY(hip_status(sr::launch_bin_and_sort(cfg, N, Vc, tiles, groups, dc, rect, tt, dk, ws + L.bin, cap,
                                              count_only ? nullptr : (uint32_t*)(ws + L.vals), nullptr,
                                              (uint32_t*)(ws + L.ranges), counters, ctx->status, count_only, s),
                      "prune pass: binning"));
    *tiles_out = tiles;
    return SR_OK;
}

sr_status check_prune_args(const sr_config* cfg, int prim, int N, const float* means, const float* scales,
                           const float* quats, const float* opac, int V, const sr_camera* cams_host,
                           const sr_camera* cams_dev, int vpc, uint32_t cap, const void* workspace, size_t ws_bytes,
                           PruneLayout* L) {
    SR_TRY(check_cfg(cfg));
    if (N < 0 || V < 0) return fail(SR_ERR_ARG, "N = %d, V = %d", N, V);
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, nullptr, nullptr));
    SR_TRY(prune_layout(cfg, prim, N, V, cams_host, vpc, cap, L));
    if (N > 0) { SR_NEED(means); SR_NEED(scales); SR_NEED(quats); SR_NEED(opac); }
    if (N > 0 && V > 0) {
        SR_NEED(workspace);
        if (ws_bytes < L->bytes) return fail(SR_ERR_ARG, "workspace of %zu bytes, %zu needed", ws_bytes, L->bytes);
    }
    return SR_OK;
}

}  // namespace

sr_status sr_prune_workspace_size(const sr_config* cfg, int32_t prim, int32_t N, int32_t V,
                                  const sr_camera* cams_host, int32_t views_per_chunk, uint32_t inst_capacity,
                                  size_t* bytes_host) {
    SR_TRY(check_cfg(cfg));
    SR_NEED(bytes_host);
    if (N < 0 || V < 0) return fail(SR_ERR_ARG, "N = %d, V = %d", N, V);
    if (V > 0) SR_NEED(cams_host);
    SR_TRY(check_views(cams_host, cams_host, V, cfg->tile_w, cfg->tile_h, nullptr, nullptr, nullptr));
    PruneLayout L;
    SR_TRY(prune_layout(cfg, prim, N, V, cams_host, views_per_chunk, inst_capacity, &L));
    *bytes_host = (N > 0 && V > 0) ? L.bytes : 0;
    return SR_OK;
}

sr_status sr_prune_plan(sr_ctx* ctx, const sr_config* cfg, int32_t prim, int32_t N, const float* means,
                        const float* scales, const float* quats, const float* opac, int32_t V,
                        const sr_camera* cams_host, const sr_camera* cams_dev, int32_t views_per_chunk,
                        void* workspace, size_t ws_bytes, uint32_t* inst_capacity_host, void* stream) {
    PruneLayout L;
    SR_TRY(check_prune_args(cfg, prim, N, means, scales, quats, opac, V, cams_host, cams_dev, views_per_chunk, 0,
                            workspace, ws_bytes, &L));
    SR_NEED(inst_capacity_host);
    *inst_capacity_host = 0;
    if (N == 0 || V == 0) return SR_OK;            // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    std::vector<sr_camera> hc;
    for (int k = 0; k < L.chunks; ++k) {
        const int v0 = k * views_per_chunk, v1 = std::min(V, v0 + views_per_chunk);
        int tiles = 0;
        SR_TRY(prune_chunk_bin(ctx, *cfg, prim, N, means, scales, quats, opac, cams_host, cams_dev, v0, v1, nullptr,
                               true, ws, L, 0, true, k, s, hc, &tiles));
    }
    std::vector<uint32_t> cnt((size_t)SR_COUNTERS * L.chunks);
    SR_TRY(hip_status(hipMemcpyAsync(cnt.data(), ws + L.counters, cnt.size() * sizeof(uint32_t),
                                     hipMemcpyDeviceToHost, s),
                      "sr_prune_plan: counts"));
    SR_TRY(hip_status(hipStreamSynchronize(s), "sr_prune_plan: synchronise"));
    uint32_t need = 0;
    for (int k = 0; k < L.chunks; ++k) need = std::max(need, cnt[(size_t)SR_COUNTERS * k + 1]);
    *inst_capacity_host = need;
    return SR_OK;
}

sr_status sr_prune_contrib(sr_ctx* ctx, const sr_config* cfg, int32_t prim, int32_t N, const float* means,
                           const float* scales, const float* quats, const float* opac, int32_t V,
                           const sr_camera* cams_host, const sr_camera* cams_dev, int32_t views_per_chunk,
                           float tau, uint32_t inst_capacity, void* workspace, size_t ws_bytes, uint32_t* hits,
                           float* max_alpha, float* max_weight, uint8_t* in_frustum, uint8_t* prune_mask,
                           void* stream) {
    PruneLayout L;
    SR_TRY(check_prune_args(cfg, prim, N, means, scales, quats, opac, V, cams_host, cams_dev, views_per_chunk,
                            inst_capacity, workspace, ws_bytes, &L));
    if (N > 0) { SR_NEED(hits); SR_NEED(max_alpha); SR_NEED(max_weight); }
    if (N == 0) return SR_OK;                      // nothing to enqueue
    SR_TRY(check_ctx(ctx));
    hipStream_t s = (hipStream_t)stream;
    const bool acc = (cfg->flags & SR_FLAG_ACCUMULATE) != 0;
    if (!acc) SR_TRY(clear_stats(N, hits, max_alpha, max_weight, s));
    char* ws = (char*)workspace;
    std::vector<sr_camera> hc;
    sr_config c = *cfg;
    c.flags |= SR_FLAG_ACCUMULATE;
    for (int k = 0; k < L.chunks; ++k) {
        const int v0 = k * views_per_chunk, v1 = std::min(V, v0 + views_per_chunk);
        int tiles = 0;
        SR_TRY(prune_chunk_bin(ctx, *cfg, prim, N, means, scales, quats, opac, cams_host, cams_dev, v0, v1,
                               in_frustum, acc || k > 0, ws, L, inst_capacity, false, k, s, hc, &tiles));
        const sr_camera* dc = (const sr_camera*)(ws + L.cams);
        const uint32_t* vals = (const uint32_t*)(ws + L.vals);
        const uint32_t* ranges = (const uint32_t*)(ws + L.ranges);
        if (prim == SR_PRIM_SURFEL)
            SR_TRY(hip_status(sr::launch_render_fwd(c, N, v1 - v0, tiles, dc, (const float*)(ws + L.geom), nullptr,
                                                    (const uint16_t*)(ws + L.rect), vals, ranges, nullptr, nullptr,
                                                    nullptr, nullptr, nullptr, nullptr, nullptr, hits, max_alpha,
                                                    max_weight, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                    ctx->status, s),
                              "prune pass: statistics"));
        else
            SR_TRY(hip_status(sr::launch_prune3d(c, N, v1 - v0, tiles, dc, (const float*)(ws + L.geom), vals, ranges,
                                                 hits, max_alpha, max_weight, ctx->status, s),
                              "prune pass: statistics"));
    }
    if (prune_mask)
        SR_TRY(hip_status(sr::launch_prune_mask(N, max_alpha, tau, ctx->status, prune_mask, s), "prune pass: mask"));
    return SR_OK;
}

}  // extern "C"
