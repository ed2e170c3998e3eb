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

// ---- 2DGS regularisers of the total loss (Eq. 3) ---------------------------
//   L_d,v = mean_p dist(p)
//   L_n,v = mean_p (A(p) - N(p) . N_d(p)),  N_d from central differences of
//           the camera-space points P = s ray, zero on the one-pixel border;
//           the surface depth s is D / A (0 where A = 0) or, when a median
//           depth map is given, the median depth (its gradient then goes to
//           that map and none to D)
//   L_reg = (1/V) sum_v (w_dist L_d,v + w_normal L_n,v)
// One workgroup per 32x8 pixel tile of a view: the camera-space points of
// the tile and a two-pixel halo are formed once in LDS, then the depth
// normals of the tile and a one-pixel halo with the two vectors every normal
// passes back to its neighbours' points (the gradient through n = a x b),
// then each pixel gathers its point's gradient from its four neighbours.
// Each pixel writes only its own gradients (no atomics); per-tile loss sums
// go to a per-(view, tile) slot and are reduced in a fixed order.

constexpr float kEpsNormal = 1e-12f;
constexpr int kRegTX = 32, kRegTY = 8;                 // tile; kNT threads
constexpr int kRegPX = kRegTX + 4, kRegPY = kRegTY + 4; // points: two-pixel halo
constexpr int kRegNX = kRegTX + 2, kRegNY = kRegTY + 2; // normals: one-pixel halo

__device__ __forceinline__ float3 f3sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 f3cross(float3 a, float3 b) {
#pragma clang fp contract(off)
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float f3dot(float3 a, float3 b) {
#pragma clang fp contract(off)
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

__host__ __device__ inline int reg_tiles_of(int W, int H) {
    return ((W + kRegTX - 1) / kRegTX) * ((H + kRegTY - 1) / kRegTY);
}
__device__ __forceinline__ int reg_tiles(int W, int H) { return reg_tiles_of(W, H); }

__global__ void __launch_bounds__(kNT)
k_reg_partial(const sr_camera* __restrict__ cams, int V, const float* __restrict__ alpha,
              const float* __restrict__ depth, const float* __restrict__ normal, const float* __restrict__ dist,
              const float* __restrict__ median, float w_dist, float w_normal, int nslot, float* __restrict__ partial,
              float* __restrict__ dL_dalpha, float* __restrict__ dL_ddepth, float* __restrict__ dL_dnormal,
              float* __restrict__ dL_ddist, float* __restrict__ dL_dmedian) {
#pragma clang fp contract(off)
    __shared__ float s[kNT];
    __shared__ float3 sP[kRegPY][kRegPX];
    __shared__ float3 sGa[kRegNY][kRegNX], sGb[kRegNY][kRegNX], sNd[kRegNY][kRegNX];
    // one flat grid over the tiles of all views
    int v = 0, tile = (int)blockIdx.x;
    for (; v < V; ++v) {
        const int nt = reg_tiles(cams[v].width, cams[v].height);
        if (tile < nt) break;
        tile -= nt;
    }
    if (v >= V) return;                                     // uniform: the whole block leaves
    const sr_camera& c = cams[v];
    const int W = c.width, H = c.height;
    const int ntx = (W + kRegTX - 1) / kRegTX;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    const int x0 = tx * kRegTX, y0 = ty * kRegTY;
    const int64_t HW = (int64_t)W * H;
    const float* A = alpha + c.pix_offset;
    const float* D = depth + c.pix_offset;
    const float* Md = median ? median + c.pix_offset : nullptr;
    const float* Nr = normal + 3 * c.pix_offset;
    const float scale = 1.0f / ((float)HW * (float)V);
    const float gn = w_normal * scale;
    const float fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
    // points P = s ray of the tile and a two-pixel halo (0 outside)
    for (int k = threadIdx.x; k < kRegPX * kRegPY; k += kNT) {
        const int ly = k / kRegPX, lx = k - ly * kRegPX;
        const int i = x0 - 2 + lx, j = y0 - 2 + ly;
        float3 P = make_float3(0.f, 0.f, 0.f);
        if (i >= 0 && i < W && j >= 0 && j < H) {
            const int64_t p = (int64_t)j * W + i;
            float sd;
            if (Md) {
                sd = Md[p];
            } else {
                const float a = A[p];
                sd = a > 0.f ? D[p] / a : 0.f;
            }
            P = make_float3(sd * (((float)i + 0.5f - cx) / fx), sd * (((float)j + 0.5f - cy) / fy), sd);
        }
        sP[ly][lx] = P;
    }
    __syncthreads();
    // depth normals of the tile and a one-pixel halo; the vectors b x dn and
    // dn x a that each normal sends to the points of its neighbours
    for (int k = threadIdx.x; k < kRegNX * kRegNY; k += kNT) {
        const int ly = k / kRegNX, lx = k - ly * kRegNX;
        const int i = x0 - 1 + lx, j = y0 - 1 + ly;
        float3 nd = make_float3(0.f, 0.f, 0.f), ga = nd, gb = nd;
        if (i >= 1 && i <= W - 2 && j >= 1 && j <= H - 2) {
            const int px = lx + 1, py = ly + 1;              // position in sP
            const float3 a = f3sub(sP[py + 1][px], sP[py - 1][px]);
            const float3 b = f3sub(sP[py][px + 1], sP[py][px - 1]);
            const float3 n = f3cross(a, b);
            const float len = sqrtf(f3dot(n, n));
            const float den = len > kEpsNormal ? len : kEpsNormal;
            nd = make_float3(n.x / den, n.y / den, n.z / den);
            const int64_t p = (int64_t)j * W + i;
            const float3 g = make_float3(-gn * Nr[p], -gn * Nr[p + HW], -gn * Nr[p + 2 * HW]);
            float3 dn;
            if (len > kEpsNormal) {
                const float kk = f3dot(nd, g);
                dn = make_float3((g.x - nd.x * kk) / len, (g.y - nd.y * kk) / len, (g.z - nd.z * kk) / len);
            } else {
                dn = make_float3(g.x / kEpsNormal, g.y / kEpsNormal, g.z / kEpsNormal);
            }
            ga = f3cross(b, dn);                             // dL/da
            gb = f3cross(dn, a);                             // dL/db
        }
        sNd[ly][lx] = nd;
        sGa[ly][lx] = ga;
        sGb[ly][lx] = gb;
    }
    __syncthreads();
    // one pixel per thread
    const int lx = (int)threadIdx.x % kRegTX, ly = (int)threadIdx.x / kRegTX;
    const int i = x0 + lx, j = y0 + ly;
    float ld = 0.f, ln = 0.f;
    if (i < W && j < H) {
        const int64_t p = (int64_t)j * W + i;
        const int64_t o1 = c.pix_offset + p, o3 = 3 * c.pix_offset + p;
        const int nx = lx + 1, ny = ly + 1;                  // position in the normal arrays
        const float3 nd = sNd[ny][nx];
        const float a = A[p];
        const float3 N = make_float3(Nr[p], Nr[p + HW], Nr[p + 2 * HW]);
        ld = dist[o1];
        ln = a - f3dot(N, nd);
        // this point is P(i, j+1) of the normal above, P(i, j-1) of the one
        // below, P(i+1, j) of the left one and P(i-1, j) of the right one
        const float3 u = sGa[ny - 1][nx], dw = sGa[ny + 1][nx], l = sGb[ny][nx - 1], r = sGb[ny][nx + 1];
        const float3 dP = make_float3(((u.x - dw.x) + l.x) - r.x, ((u.y - dw.y) + l.y) - r.y,
                                      ((u.z - dw.z) + l.z) - r.z);
        const float3 ray = make_float3(((float)i + 0.5f - cx) / fx, ((float)j + 0.5f - cy) / fy, 1.0f);
        const float ds = f3dot(dP, ray);
        float gA = gn, gD = 0.f;
        if (Md) {
            dL_dmedian[o1] = ds;
        } else if (a > 0.f) {
            gD = ds / a;
            gA = gA - ds * (D[p] / a) / a;
        }
        dL_dalpha[o1] += gA;
        dL_ddepth[o1] = gD;
        dL_dnormal[o3] = -gn * nd.x;
        dL_dnormal[o3 + HW] = -gn * nd.y;
        dL_dnormal[o3 + 2 * HW] = -gn * nd.z;
        dL_ddist[o1] = w_dist * scale;
    }
    ld = block_sum(ld, s);
    ln = block_sum(ln, s);
    if (threadIdx.x == 0) {
        partial[2 * ((size_t)v * nslot + tile)] = ld;
        partial[2 * ((size_t)v * nslot + tile) + 1] = ln;
    }
}

// loss[v] = L_d,v, loss[V+v] = L_n,v from the chunk partials; loss[2V] total
__global__ void __launch_bounds__(kNT)
k_reg_final(const sr_camera* __restrict__ cams, int V, int nslot, const float* __restrict__ partial,
            float* __restrict__ loss) {
    __shared__ float s[kNT];
    const int v = blockIdx.x;
    const int nt = reg_tiles(cams[v].width, cams[v].height);
    float ld = 0.f, ln = 0.f;
    for (int i = threadIdx.x; i < nt; i += kNT) {
        ld += partial[2 * ((size_t)v * nslot + i)];
        ln += partial[2 * ((size_t)v * nslot + i) + 1];
    }
    ld = block_sum(ld, s);
    ln = block_sum(ln, s);
    if (threadIdx.x == 0) {
        const float HW = (float)cams[v].width * (float)cams[v].height;
        loss[v] = ld / HW;
        loss[V + v] = ln / HW;
    }
}

__global__ void __launch_bounds__(kNT)
k_reg_total(int V, float w_dist, float w_normal, float* __restrict__ loss) {
    __shared__ float s[kNT];
    float t = 0.f;
    for (int v = threadIdx.x; v < V; v += kNT) t += w_dist * loss[v] + w_normal * loss[V + v];
    t = block_sum(t, s);
    if (threadIdx.x == 0) loss[2 * V] = t / (float)V;
}

}  // namespace

int reg_tile_count(int W, int H) { return reg_tiles_of(W, H); }

hipError_t launch_reg_loss(int V, int max_tiles, int total_tiles, const sr_camera* cams, const float* alpha,
                           const float* depth,
                           const float* normal, const float* dist, const float* median, float w_dist,
                           float w_normal, void* ws, float* loss, float* dL_dalpha, float* dL_ddepth,
                           float* dL_dnormal, float* dL_ddist, float* dL_dmedian, hipStream_t s) {
    if (V == 0 || max_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reg_partial, dim3(total_tiles), dim3(kNT), 0, s, cams, V, alpha, depth, normal, dist,
                       median, w_dist, w_normal, max_tiles, (float*)ws, dL_dalpha, dL_ddepth, dL_dnormal, dL_ddist,
                       dL_dmedian);
    hipLaunchKernelGGL(k_reg_final, dim3(V), dim3(kNT), 0, s, cams, V, max_tiles, (const float*)ws, loss);
    hipLaunchKernelGGL(k_reg_total, dim3(1), dim3(kNT), 0, s, V, w_dist, w_normal, loss);
    return hipGetLastError();
}

hipError_t launch_loss_from_tiles(int V, const sr_camera* cams, const float* tile_loss, float gamma, float w_c,
                                  float* loss, hipStream_t s) {
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss_tiles, dim3(V), dim3(kNT), 0, s, cams, V, tile_loss, loss);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(kNT), 0, s, V, gamma, w_c, loss);
    return hipGetLastError();
}

int loss_chunks(int64_t max_hw) { return (int)((max_hw + kChunk - 1) / kChunk); }

size_t loss_workspace_bytes(int V, int64_t max_hw, int max_reg_tiles) {
    const int64_t slots = loss_chunks(max_hw) > max_reg_tiles ? loss_chunks(max_hw) : max_reg_tiles;
    return (size_t)V * (size_t)slots * 2 * sizeof(float);
}

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
