// C ABI of the surfel rasterizer: host-side argument validation and
// dispatch to the HIP kernels.  No entry point allocates device memory or
// synchronises; every launch goes to the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "launch.h"
#include "surfelrast.h"

static_assert(sizeof(sr_camera) == 128, "sr_camera must stay 128 bytes");

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

int32_t sr_version(void) { return 1; }

int32_t sr_tile_supported(int32_t tile_w, int32_t tile_h) { return sr::tile_shape_supported(tile_w, tile_h) ? 1 : 0; }

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

sr_status sr_preprocess(const sr_config* cfg, int32_t N, const float* means, const float* scales,
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

sr_status sr_bin_and_sort(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
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
    return hip_status(sr::launch_bin_and_sort(*cfg, N, V, total_tiles, total_groups, cams_dev, rect, tiles_touched,
                                              depth_key,
                                              workspace, inst_capacity, vals, keys64, ranges, counters,
                                              (hipStream_t)stream),
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

sr_status sr_render_forward(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
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
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE)) SR_TRY(clear_stats(N, hits, max_alpha, max_weight, s));
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, app, nullptr, vals, ranges,
                                            color, alpha, depth, normal, dist, T_final, n_contrib, hits, max_alpha,
                                            max_weight, nullptr, median_depth, median_contrib, tile_order,
                                            tile_cost, s),
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

sr_status sr_backward_raster(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                             const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                             const uint32_t* ranges, const float* alpha, const float* depth, const float* dist,
                             const float* T_final, const uint32_t* n_contrib, const float* dL_dcolor,
                             const float* dL_dalpha, const float* dL_ddepth, const float* dL_dnormal,
                             const float* dL_ddist, const uint32_t* median_contrib, const float* dL_dmedian,
                             float* grad_rec, const uint32_t* tile_order, void* stream) {
    int total_tiles = 0;
    SR_TRY(check_backward_raster(cfg, N, V, cams_host, cams_dev, geom, app, vals, ranges, alpha, depth, dist, T_final,
                                 n_contrib, grad_rec, &total_tiles));
    if (dL_dmedian && !median_contrib) return fail(SR_ERR_ARG, "dL_dmedian needs median_contrib");
    if (N == 0 || V == 0) return SR_OK;
    return hip_status(sr::launch_render_bwd(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, alpha, depth,
                                            dist, T_final, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dnormal,
                                            dL_ddist, median_contrib, dL_dmedian, grad_rec, tile_order,
                                            (hipStream_t)stream),
                      "sr_backward_raster");
}

sr_status sr_backward_project(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                              const sr_camera* cams_dev, const float* means, const float* scales, const float* quats,
                              const float* sh, const float* geom, const float* app, const uint32_t* tiles_touched,
                              float* grad_rec, float* g_means, float* g_scales, float* g_quats, float* g_opac,
                              float* g_sh, float* densify_grad, uint32_t* densify_count, void* stream) {
    SR_TRY(check_backward_project(cfg, N, V, cams_host, cams_dev, means, scales, quats, sh, geom, app, grad_rec,
                                  g_means, g_scales, g_quats, g_opac, g_sh));
    if ((densify_grad || densify_count) && !tiles_touched)
        return fail(SR_ERR_ARG, "the density statistics need tiles_touched (the views each surfel is seen in)");
    if (N == 0 || V == 0) return SR_OK;
    return hip_status(sr::launch_preprocess_bwd(*cfg, N, means, scales, quats, sh, V, cams_dev, geom, app,
                                                tiles_touched, grad_rec, g_means, g_scales, g_quats, g_opac, g_sh,
                                                densify_grad, densify_count, (hipStream_t)stream),
                      "sr_backward_project");
}

sr_status sr_render_backward(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
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
    hipStream_t s = (hipStream_t)stream;
    SR_TRY(hip_status(sr::fill_f32(grad_rec, 0.f, (uint64_t)V * N * SR_GRAD_STRIDE, s), "clear grad_rec"));
    SR_TRY(hip_status(sr::launch_render_bwd(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, alpha, depth,
                                            dist, T_final, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dnormal,
                                            dL_ddist, median_contrib, dL_dmedian, grad_rec, nullptr, s),
                      "render backward"));
    return hip_status(sr::launch_preprocess_bwd(*cfg, N, means, scales, quats, sh, V, cams_dev, geom, app, nullptr,
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

sr_status sr_background_loss(int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* alpha,
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
    return hip_status(sr::launch_loss(V, mhw, cams_dev, alpha, mask, color, target, gamma, w_c, workspace, loss,
                                      dL_dalpha, dL_dcolor, (hipStream_t)stream),
                      "sr_background_loss");
}

sr_status sr_regularizer_loss(int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* alpha,
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

sr_status sr_ssim_loss(int32_t V, const sr_camera* cams_host, const sr_camera* cams_dev, const float* color,
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
    return hip_status(sr::launch_ssim(V, ms, tot, P, cams_dev, color, target, mask, w_s, workspace, out, dL_dcolor,
                                      (hipStream_t)stream),
                      "sr_ssim_loss");
}

sr_status sr_preprocess_3d(const sr_config* cfg, int32_t N, const float* means, const float* scales,
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
    return hip_status(sr::launch_preprocess3d(*cfg, N, means, scales, quats, opac, V, cams_dev, geom3, rect,
                                              tiles_touched, depth_key, in_frustum, (hipStream_t)stream),
                      "sr_preprocess_3d");
}

sr_status sr_prune_contrib_3d(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                              const sr_camera* cams_dev, const float* geom3, const uint32_t* vals,
                              const uint32_t* ranges, uint32_t* hits, float* max_alpha, float* max_weight,
                              void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (N > 0) { SR_NEED(hits); SR_NEED(max_alpha); SR_NEED(max_weight); }
    if (total_tiles > 0) { SR_NEED(geom3); SR_NEED(vals); SR_NEED(ranges); }
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE) && N > 0) {
        SR_TRY(hip_status(sr::fill_f32((float*)hits, 0.f, (uint64_t)N, s), "clear hits"));
        SR_TRY(hip_status(sr::fill_f32(max_alpha, 0.f, (uint64_t)N, s), "clear max_alpha"));
        SR_TRY(hip_status(sr::fill_f32(max_weight, 0.f, (uint64_t)N, s), "clear max_weight"));
    }
    return hip_status(sr::launch_prune3d(*cfg, N, V, total_tiles, cams_dev, geom3, vals, ranges, hits, max_alpha,
                                         max_weight, s),
                      "sr_prune_contrib_3d");
}

sr_status sr_compact_workspace_size(int32_t N, size_t* bytes_host) {
    if (N < 0) return fail(SR_ERR_ARG, "N < 0");
    SR_NEED(bytes_host);
    *bytes_host = sr::compact_workspace_bytes(N);
    return SR_OK;
}

sr_status sr_compact_surfels(int32_t N, const uint8_t* prune_mask, const float* opac, float min_opacity,
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
    return hip_status(sr::launch_compact(N, prune_mask, opac, min_opacity, n_arrays, src_host, dst_host,
                                         (const int*)widths_host, workspace, n_kept, (hipStream_t)stream),
                      "sr_compact_surfels");
}

sr_status sr_prune_contrib(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                           const sr_camera* cams_dev, const float* geom, const uint16_t* rect, const uint32_t* vals,
                           const uint32_t* ranges, uint32_t* hits, float* max_alpha, float* max_weight,
                           void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (N > 0) { SR_NEED(hits); SR_NEED(max_alpha); SR_NEED(max_weight); }
    if (total_tiles > 0) { SR_NEED(geom); SR_NEED(vals); SR_NEED(ranges); }
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE) && N > 0) {
        SR_TRY(hip_status(sr::fill_f32((float*)hits, 0.f, (uint64_t)N, s), "clear hits"));
        SR_TRY(hip_status(sr::fill_f32(max_alpha, 0.f, (uint64_t)N, s), "clear max_alpha"));
        SR_TRY(hip_status(sr::fill_f32(max_weight, 0.f, (uint64_t)N, s), "clear max_weight"));
    }
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, nullptr, rect, vals, ranges,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, hits,
                                            max_alpha, max_weight, nullptr, nullptr, nullptr, nullptr, nullptr, s),
                      "sr_prune_contrib");
}

sr_status sr_train_step_raster(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                               const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                               const uint32_t* ranges, const uint8_t* mask, const float* target, float gamma,
                               float w_c, float* color, float* alpha, float* depth, float* normal, float* dist,
                               float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha,
                               float* max_weight, float* tile_loss, float* loss, float* grad_rec,
                               const uint32_t* tile_order, uint32_t* tile_cost, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    if (total_tiles > 0) {
        SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges); SR_NEED(mask); SR_NEED(target);
        SR_NEED(color); SR_NEED(alpha); SR_NEED(depth); SR_NEED(normal); SR_NEED(dist); SR_NEED(T_final);
        SR_NEED(n_contrib); SR_NEED(tile_loss); SR_NEED(loss); SR_NEED(grad_rec);
    }
    SR_TRY(check_stats(hits, max_alpha, max_weight));
    hipStream_t s = (hipStream_t)stream;
    if (!(cfg->flags & SR_FLAG_ACCUMULATE)) SR_TRY(clear_stats(N, hits, max_alpha, max_weight, s));
    if (total_tiles == 0) return SR_OK;
    SR_TRY(hip_status(sr::launch_train_raster(*cfg, N, V, total_tiles, cams_dev, geom, app, vals, ranges, mask, target,
                                              gamma, w_c, color, alpha, depth, normal, dist, T_final, n_contrib, hits,
                                              max_alpha, max_weight, tile_loss, grad_rec, tile_order, tile_cost, s),
                      "sr_train_step_raster"));
    return hip_status(sr::launch_loss_from_tiles(V, cams_dev, tile_loss, gamma, w_c, loss, s), "loss totals");
}

sr_status sr_render_count(const sr_config* cfg, int32_t N, int32_t V, const sr_camera* cams_host,
                          const sr_camera* cams_dev, const float* geom, const float* app, const uint32_t* vals,
                          const uint32_t* ranges, uint64_t* counts, void* stream) {
    SR_TRY(check_cfg(cfg));
    SR_TRY(check_nv(N, V));
    int total_tiles = 0;
    SR_TRY(check_views(cams_host, cams_dev, V, cfg->tile_w, cfg->tile_h, nullptr, &total_tiles, nullptr));
    SR_NEED(counts);
    if (total_tiles > 0) { SR_NEED(geom); SR_NEED(app); SR_NEED(vals); SR_NEED(ranges); }
    hipStream_t s = (hipStream_t)stream;
    SR_TRY(hip_status(sr::fill_f32((float*)counts, 0.f, 10, s), "clear counts"));
    return hip_status(sr::launch_render_fwd(*cfg, N, V, total_tiles, cams_dev, geom, app, nullptr, vals, ranges,
                                            nullptr,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                            nullptr, (unsigned long long*)counts, nullptr, nullptr, nullptr, nullptr,
                                            s),
                      "sr_render_count");
}

sr_status sr_prune_mask(int32_t N, const float* max_alpha, float tau, uint8_t* prune_mask, void* stream) {
    if (N < 0) return fail(SR_ERR_ARG, "N < 0");
    if (N > 0) { SR_NEED(max_alpha); SR_NEED(prune_mask); }
    return hip_status(sr::launch_prune_mask(N, max_alpha, tau, prune_mask, (hipStream_t)stream), "sr_prune_mask");
}

sr_status sr_tile_order_workspace_size(int32_t T, size_t* bytes_host) {
    if (T < 0) return fail(SR_ERR_ARG, "T = %d < 0", T);
    SR_NEED(bytes_host);
    *bytes_host = T > 0 ? sr::tile_order_workspace(T) : 0;
    return SR_OK;
}

sr_status sr_tile_order(int32_t T, const uint32_t* tile_cost, void* workspace, size_t ws_bytes,
                        uint32_t* tile_order, void* stream) {
    if (T < 0) return fail(SR_ERR_ARG, "T = %d < 0", T);
    if (T == 0) return SR_OK;
    SR_NEED(tile_cost); SR_NEED(workspace); SR_NEED(tile_order);
    if (ws_bytes < sr::tile_order_workspace(T))
        return fail(SR_ERR_ARG, "workspace of %zu bytes < %zu", ws_bytes, sr::tile_order_workspace(T));
    return hip_status(sr::launch_tile_order(T, tile_cost, workspace, tile_order, (hipStream_t)stream),
                      "sr_tile_order");
}

}  // extern "C"
