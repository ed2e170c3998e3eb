// Masked losses on the rendered views (Section 4.2):
//   background loss (Eq. 1)   L_b,v = (1/(H W)) sum_p A(p) (1 - M(p))
//   masked photometric L1 (Eq. 2, L1 part)  L1_v = (1/(3 H W)) sum |M C - M I|
// and the gradients of L = (1/V) sum_v (w_c L1_v + gamma L_b,v).
// Per-view sums use a fixed two-stage reduction order (deterministic).
#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr int kNT = 256;
constexpr int kChunk = 8192;   // pixels per block of the first stage

__device__ __forceinline__ float block_sum(float v, float* s) {
    // fixed-order tree over the 256 threads
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = kNT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const float r = s[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kNT)
k_loss_partial(const sr_camera* __restrict__ cams, int V, const float* __restrict__ alpha,
               const uint8_t* __restrict__ mask, const float* __restrict__ color, const float* __restrict__ target,
               float gamma, float w_c, int nchunk, float* __restrict__ partial, float* __restrict__ dL_dalpha,
               float* __restrict__ dL_dcolor) {
    __shared__ float s[kNT];
    const int v = blockIdx.y;
    const sr_camera& c = cams[v];
    const int64_t HW = (int64_t)c.width * c.height;
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    float lb = 0.f, l1 = 0.f;
    if (b < HW) {
        const int64_t e = b + kChunk < HW ? b + kChunk : HW;
        for (int64_t p = b + threadIdx.x; p < e; p += kNT) {
            const int64_t o1 = c.pix_offset + p;
            const int64_t o3 = 3 * c.pix_offset + p;
            float C[3] = {0.f, 0.f, 0.f}, I[3] = {0.f, 0.f, 0.f}, gC[3], gA;
            if (color) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    C[ch] = color[o3 + ch * HW];
                    I[ch] = target[o3 + ch * HW];
                }
            }
            float l1p = 0.f;
            pixel_loss_grad(mask[o1], alpha[o1], C, I, gamma, w_c, (float)HW, (float)V, lb, l1p, gA, gC);
            if (dL_dalpha) dL_dalpha[o1] = gA;
            if (color) {
                l1 += l1p;
                if (dL_dcolor) {
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) dL_dcolor[o3 + ch * HW] = gC[ch];
                }
            }
        }
    }
    lb = block_sum(lb, s);
    l1 = block_sum(l1, s);
    if (threadIdx.x == 0) {
        partial[2 * ((size_t)v * nchunk + blockIdx.x)] = lb;
        partial[2 * ((size_t)v * nchunk + blockIdx.x) + 1] = l1;
    }
}

__global__ void __launch_bounds__(kNT)
k_loss_final(const sr_camera* __restrict__ cams, int V, int nchunk, const float* __restrict__ partial,
             float* __restrict__ loss) {
    __shared__ float s[kNT];
    const int v = blockIdx.x;
    float lb = 0.f, l1 = 0.f;
    for (int i = threadIdx.x; i < nchunk; i += kNT) {
        lb += partial[2 * ((size_t)v * nchunk + i)];
        l1 += partial[2 * ((size_t)v * nchunk + i) + 1];
    }
    lb = block_sum(lb, s);
    l1 = block_sum(l1, s);
    if (threadIdx.x == 0) {
        const float HW = (float)cams[v].width * (float)cams[v].height;
        loss[v] = lb / HW;
        loss[V + v] = l1 / (3.0f * HW);
    }
}

// loss[2V] = (1/V) sum_v (w_c L1_v + gamma L_b,v), summed in view order
__global__ void __launch_bounds__(kNT)
k_loss_total(int V, float gamma, float w_c, float* __restrict__ loss) {
    __shared__ float s[kNT];
    float t = 0.f;
    for (int v = threadIdx.x; v < V; v += kNT) t += w_c * loss[V + v] + gamma * loss[v];
    t = block_sum(t, s);
    if (threadIdx.x == 0) loss[2 * V] = t / (float)V;
}

// Per-view totals from the per-tile partial sums of the fused training step
// (tiles of a view are contiguous), summed in tile order.
__global__ void __launch_bounds__(kNT)
k_loss_tiles(const sr_camera* __restrict__ cams, int V, const float* __restrict__ tile_loss,
             float* __restrict__ loss) {
    __shared__ float s[kNT];
    const int v = blockIdx.x;
    const sr_camera& c = cams[v];
    const int T0 = c.tile_offset, nt = c.tiles_x * c.tiles_y;
    float lb = 0.f, l1 = 0.f;
    for (int i = threadIdx.x; i < nt; i += kNT) {
        lb += tile_loss[2 * (size_t)(T0 + i)];
        l1 += tile_loss[2 * (size_t)(T0 + i) + 1];
    }
    lb = block_sum(lb, s);
    l1 = block_sum(l1, s);
    if (threadIdx.x == 0) {
        const float HW = (float)c.width * (float)c.height;
        loss[v] = lb / HW;
        loss[V + v] = l1 / (3.0f * HW);
    }
}

}  // namespace

hipError_t launch_loss_from_tiles(int V, const sr_camera* cams, const float* tile_loss, float gamma, float w_c,
                                  float* loss, hipStream_t s) {
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss_tiles, dim3(V), dim3(kNT), 0, s, cams, V, tile_loss, loss);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(kNT), 0, s, V, gamma, w_c, loss);
    return hipGetLastError();
}

int loss_chunks(int64_t max_hw) { return (int)((max_hw + kChunk - 1) / kChunk); }

size_t loss_workspace_bytes(int V, int64_t max_hw) { return (size_t)V * loss_chunks(max_hw) * 2 * sizeof(float); }

hipError_t launch_loss(int V, int64_t max_hw, const sr_camera* cams, const float* alpha, const uint8_t* mask,
                       const float* color, const float* target, float gamma, float w_c, void* ws, float* loss,
                       float* dL_dalpha, float* dL_dcolor, hipStream_t s) {
    if (V == 0) return hipSuccess;
    const int nchunk = loss_chunks(max_hw);
    hipLaunchKernelGGL(k_loss_partial, dim3(nchunk, V), dim3(kNT), 0, s, cams, V, alpha, mask, color, target, gamma,
                       w_c, nchunk, (float*)ws, dL_dalpha, dL_dcolor);
    hipLaunchKernelGGL(k_loss_final, dim3(V), dim3(kNT), 0, s, cams, V, nchunk, (const float*)ws, loss);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(kNT), 0, s, V, gamma, color ? w_c : 0.f, loss);
    return hipGetLastError();
}

}  // namespace sr
