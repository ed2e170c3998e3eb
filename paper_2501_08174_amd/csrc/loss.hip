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
//           the camera-space points P = (D / A) ray (0 where A = 0), zero on
//           the one-pixel border
//   L_reg = (1/V) sum_v (w_dist L_d,v + w_normal L_n,v)
// Every pixel computes its own depth normal and, by gathering, the gradient
// that its point receives through the depth normals of its four neighbours
// (no atomics: each pixel writes only its own gradients).

constexpr float kEpsNormal = 1e-12f;

struct RegView {
    const float* A;
    const float* D;
    int W, H;
    float fx, fy, cx, cy;
};

__device__ __forceinline__ float3 reg_ray(const RegView& r, int i, int j) {
#pragma clang fp contract(off)
    return make_float3(((float)i + 0.5f - r.cx) / r.fx, ((float)j + 0.5f - r.cy) / r.fy, 1.0f);
}

__device__ __forceinline__ float3 reg_point(const RegView& r, int i, int j) {
#pragma clang fp contract(off)
    const int64_t p = (int64_t)j * r.W + i;
    const float a = r.A[p];
    const float s = a > 0.f ? r.D[p] / a : 0.f;
    const float3 ray = reg_ray(r, i, j);
    return make_float3(s * ray.x, s * ray.y, s * ray.z);
}

__device__ __forceinline__ float3 f3sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 f3cross(float3 a, float3 b) {
#pragma clang fp contract(off)
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float f3dot(float3 a, float3 b) {
#pragma clang fp contract(off)
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

__device__ __forceinline__ bool reg_interior(const RegView& r, int i, int j) {
    return i >= 1 && i <= r.W - 2 && j >= 1 && j <= r.H - 2;
}

// Depth normal of an interior pixel: the difference vectors a (rows), b
// (columns), the unnormalised normal length and N_d.
struct DepthNormal {
    float3 a, b, nd;
    float len;
};

__device__ __forceinline__ DepthNormal reg_depth_normal(const RegView& r, int i, int j) {
#pragma clang fp contract(off)
    DepthNormal d;
    d.a = f3sub(reg_point(r, i, j + 1), reg_point(r, i, j - 1));
    d.b = f3sub(reg_point(r, i + 1, j), reg_point(r, i - 1, j));
    const float3 n = f3cross(d.a, d.b);
    d.len = sqrtf(f3dot(n, n));
    const float den = d.len > kEpsNormal ? d.len : kEpsNormal;
    d.nd = make_float3(n.x / den, n.y / den, n.z / den);
    return d;
}

// Gradient of the loss with respect to the unnormalised normal n, given the
// gradient g with respect to N_d = n / max(|n|, eps).
__device__ __forceinline__ float3 reg_dn(const DepthNormal& d, float3 g) {
#pragma clang fp contract(off)
    if (d.len > kEpsNormal) {
        const float k = f3dot(d.nd, g);
        return make_float3((g.x - d.nd.x * k) / d.len, (g.y - d.nd.y * k) / d.len, (g.z - d.nd.z * k) / d.len);
    }
    return make_float3(g.x / kEpsNormal, g.y / kEpsNormal, g.z / kEpsNormal);
}

__global__ void __launch_bounds__(kNT)
k_reg_partial(const sr_camera* __restrict__ cams, int V, const float* __restrict__ alpha,
              const float* __restrict__ depth, const float* __restrict__ normal, const float* __restrict__ dist,
              float w_dist, float w_normal, int nchunk, float* __restrict__ partial, float* __restrict__ dL_dalpha,
              float* __restrict__ dL_ddepth, float* __restrict__ dL_dnormal, float* __restrict__ dL_ddist) {
#pragma clang fp contract(off)
    __shared__ float s[kNT];
    const int v = blockIdx.y;
    const sr_camera& c = cams[v];
    const int64_t HW = (int64_t)c.width * c.height;
    RegView r;
    r.A = alpha + c.pix_offset;
    r.D = depth + c.pix_offset;
    r.W = c.width; r.H = c.height;
    r.fx = c.fx; r.fy = c.fy; r.cx = c.cx; r.cy = c.cy;
    const float* Nr = normal + 3 * c.pix_offset;
    const float scale = 1.0f / ((float)HW * (float)V);
    const float gn = w_normal * scale;
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    float ld = 0.f, ln = 0.f;
    if (b < HW) {
        const int64_t e = b + kChunk < HW ? b + kChunk : HW;
        for (int64_t p = b + threadIdx.x; p < e; p += kNT) {
            const int j = (int)(p / r.W), i = (int)(p - (int64_t)j * r.W);
            const int64_t o1 = c.pix_offset + p, o3 = 3 * c.pix_offset + p;
            const float A = r.A[p];
            const float3 N = make_float3(Nr[p], Nr[p + HW], Nr[p + 2 * HW]);
            float3 nd = make_float3(0.f, 0.f, 0.f);
            if (reg_interior(r, i, j)) nd = reg_depth_normal(r, i, j).nd;
            ld += dist[o1];
            ln += A - f3dot(N, nd);
            // gradient of the point of this pixel through its neighbours' normals
            float3 dP = make_float3(0.f, 0.f, 0.f);
            const int ni[4] = {i, i, i - 1, i + 1}, nj[4] = {j - 1, j + 1, j, j};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!reg_interior(r, ni[q], nj[q])) continue;
                const DepthNormal d = reg_depth_normal(r, ni[q], nj[q]);
                const int64_t pq = (int64_t)nj[q] * r.W + ni[q];
                const float3 g = make_float3(-gn * Nr[pq], -gn * Nr[pq + HW], -gn * Nr[pq + 2 * HW]);
                const float3 dn = reg_dn(d, g);
                // n = a x b: dL/da = b x dn, dL/db = dn x a
                const float3 t = q < 2 ? f3cross(d.b, dn) : f3cross(dn, d.a);
                const float sg = (q == 0 || q == 2) ? 1.0f : -1.0f;
                dP = make_float3(dP.x + sg * t.x, dP.y + sg * t.y, dP.z + sg * t.z);
            }
            const float3 ray = reg_ray(r, i, j);
            const float ds = f3dot(dP, ray);
            float gA = gn, gD = 0.f;
            if (A > 0.f) {
                gD = ds / A;
                gA = gA - ds * (r.D[p] / A) / A;
            }
            dL_dalpha[o1] += gA;
            dL_ddepth[o1] = gD;
            dL_dnormal[o3] = -gn * nd.x;
            dL_dnormal[o3 + HW] = -gn * nd.y;
            dL_dnormal[o3 + 2 * HW] = -gn * nd.z;
            dL_ddist[o1] = w_dist * scale;
        }
    }
    ld = block_sum(ld, s);
    ln = block_sum(ln, s);
    if (threadIdx.x == 0) {
        partial[2 * ((size_t)v * nchunk + blockIdx.x)] = ld;
        partial[2 * ((size_t)v * nchunk + blockIdx.x) + 1] = ln;
    }
}

// loss[v] = L_d,v, loss[V+v] = L_n,v from the chunk partials; loss[2V] total
__global__ void __launch_bounds__(kNT)
k_reg_final(const sr_camera* __restrict__ cams, int V, int nchunk, const float* __restrict__ partial,
            float* __restrict__ loss) {
    __shared__ float s[kNT];
    const int v = blockIdx.x;
    float ld = 0.f, ln = 0.f;
    for (int i = threadIdx.x; i < nchunk; i += kNT) {
        ld += partial[2 * ((size_t)v * nchunk + i)];
        ln += partial[2 * ((size_t)v * nchunk + i) + 1];
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

hipError_t launch_reg_loss(int V, int64_t max_hw, const sr_camera* cams, const float* alpha, const float* depth,
                           const float* normal, const float* dist, float w_dist, float w_normal, void* ws,
                           float* loss, float* dL_dalpha, float* dL_ddepth, float* dL_dnormal, float* dL_ddist,
                           hipStream_t s) {
    if (V == 0) return hipSuccess;
    const int nchunk = loss_chunks(max_hw);
    hipLaunchKernelGGL(k_reg_partial, dim3(nchunk, V), dim3(kNT), 0, s, cams, V, alpha, depth, normal, dist, w_dist,
                       w_normal, nchunk, (float*)ws, dL_dalpha, dL_ddepth, dL_dnormal, dL_ddist);
    hipLaunchKernelGGL(k_reg_final, dim3(V), dim3(kNT), 0, s, cams, V, nchunk, (const float*)ws, loss);
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
