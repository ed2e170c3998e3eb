// Host-side launchers of the kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "surfelrast.h"

namespace sr {

hipError_t launch_preprocess(const sr_config& cfg, int N, const float* means, const float* scales,
                             const float* quats, const float* opac, const float* sh, int V,
                             const sr_camera* cams_dev, float* geom, float* app, uint16_t* rect,
                             uint32_t* tiles_touched, uint32_t* depth_key, uint8_t* in_frustum,
                             hipStream_t stream);

hipError_t launch_preprocess_bwd(const sr_config& cfg, int N, const float* means, const float* scales,
                                 const float* quats, const float* sh, int V, const sr_camera* cams_dev,
                                 const float* geom, const float* app, uint32_t* tiles_touched,
                                 float* grad_rec, float* g_means, float* g_scales, float* g_quats,
                                 float* g_opac, float* g_sh, float* dens_grad, uint32_t* dens_count,
                                 hipStream_t stream);

size_t bin_workspace_bytes(uint64_t VN, uint64_t cap);
size_t tile_order_workspace(int T);
hipError_t launch_tile_order(int T, const uint32_t* cost, void* ws, uint32_t* order, hipStream_t s);

hipError_t launch_bin_and_sort(const sr_config& cfg, int N, int V, int total_tiles, int total_groups,
                               const sr_camera* cams_dev,
                               const uint16_t* rect, const uint32_t* tiles_touched, const uint32_t* depth_key,
                               void* workspace, uint32_t cap, uint32_t* vals, uint64_t* keys64, uint32_t* ranges,
                               uint32_t* counters, uint32_t* status, bool count_only, hipStream_t s);
hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_rebase_cams(const sr_camera* src, int Vc, sr_camera* dst, hipStream_t s);

bool tile_shape_supported(int tw, int th);
// a backward batch compiled for the tile shape (0: the default one)
bool bwd_batch_supported(int tw, int th, int batch);

hipError_t fill_f32(float* p, float v, uint64_t n, hipStream_t s);

hipError_t launch_render_fwd(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                             const float* geom, const float* app, const uint16_t* rect, const uint32_t* vals,
                             const uint32_t* ranges, float* color, float* alpha, float* depth, float* normal,
                             float* dist, float* T_final,
                             uint32_t* n_contrib, uint32_t* hits, float* max_alpha, float* max_weight,
                             unsigned long long* counts, float* median_depth, uint32_t* median_contrib,
                             const uint32_t* tile_order, uint32_t* tile_cost, const uint32_t* status,
                             hipStream_t s);

hipError_t launch_render_bwd(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                             const float* geom, const float* app, const uint32_t* vals, const uint32_t* ranges,
                             const float* alpha, const float* depth, const float* dist, const float* T_final,
                             const uint32_t* n_contrib, const float* dC, const float* dA, const float* dD,
                             const float* dN, const float* dS, const uint32_t* median_contrib, const float* dMed,
                             float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order,
                             const uint32_t* status, hipStream_t s);

hipError_t launch_train_raster(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                               const float* geom, const float* app, const uint32_t* vals, const uint32_t* ranges,
                               const uint8_t* mask, const float* target, float gamma, float w_c, float* color,
                               float* alpha, float* depth, float* normal, float* dist, float* T_final,
                               uint32_t* n_contrib, uint32_t* hits, float* max_alpha, float* max_weight,
                               float* tile_loss, float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order,
                               uint32_t* tile_cost, const uint32_t* status, hipStream_t s);

// The device address of the training step's file-scope scratch array on
// `device` (which must be current at the first call for that device).
hipError_t scratch_address(int device, float** out);

hipError_t launch_loss_from_tiles(int V, const sr_camera* cams, const float* tile_loss, float gamma, float w_c,
                                  float* loss, hipStream_t s);

hipError_t launch_prune_mask(int N, const float* max_alpha, float tau, const uint32_t* status, uint8_t* mask,
                             hipStream_t s);

int loss_chunks(int64_t max_hw);
size_t loss_workspace_bytes(int V, int64_t max_hw, int max_reg_tiles);
int reg_tile_count(int W, int H);
hipError_t launch_loss(int V, int64_t max_hw, const sr_camera* cams, const float* alpha, const uint8_t* mask,
                       const float* color, const float* target, float gamma, float w_c, void* ws, float* loss,
                       float* dL_dalpha, float* dL_dcolor, hipStream_t s);
hipError_t launch_reg_loss(int V, int max_tiles, int total_tiles, const sr_camera* cams, const float* alpha,
                           const float* depth,
                           const float* normal, const float* dist, const float* median, float w_dist,
                           float w_normal, void* ws, float* loss, float* dL_dalpha, float* dL_ddepth,
                           float* dL_dnormal, float* dL_ddist, float* dL_dmedian, hipStream_t s);

hipError_t launch_preprocess3d(const sr_config& cfg, int N, const float* means, const float* scales,
                               const float* quats, const float* opac, int V, const sr_camera* cams_dev,
                               float* geom3, uint16_t* rect, uint32_t* tiles_touched, uint32_t* depth_key,
                               uint8_t* in_frustum, hipStream_t s);
hipError_t launch_prune3d(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                          const float* geom3, const uint32_t* vals, const uint32_t* ranges, uint32_t* hits,
                          float* max_alpha, float* max_weight, const uint32_t* status, hipStream_t s);
size_t compact_workspace_bytes(int N);
hipError_t launch_compact(int N, const uint8_t* prune, const float* opac, float min_opac, int n_arrays,
                          const float* const* src, float* const* dst, const int* widths, void* ws,
                          uint32_t* n_kept, hipStream_t s);
int ssim_slots(int W, int H);
size_t ssim_workspace_bytes(int V, int max_slots, int64_t P, bool with_grad);
hipError_t launch_ssim(int V, int max_slots, int total_slots, int64_t P, const sr_camera* cams, const float* color,
                       const float* target, const uint8_t* mask, float w_s, void* ws, float* out,
                       float* dL_dcolor, hipStream_t s);

}  // namespace sr
