// Masked structural similarity of the rendered and target views: the D-SSIM
// part of the photometric loss of Eq. 2 (the 3DGS loss on M*R and M*I) with
// its gradient, and the masked SSIM / PSNR metrics.
//
//   x = M R, y = M I per colour channel; G = 11x11 Gaussian (sigma 1.5,
//   normalised, separable), correlation with zero padding
//   S(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2))
//   SSIM_v = mean of S over channels and pixels; L = (1/V) sum_v w_s (1 - SSIM_v)
//   PSNR_v = -10 log10(mean (x - y)^2)
//
// Forward: per 32x16 tile and channel, x and y with a five-pixel halo go to
// LDS, a horizontal then a vertical 11-tap pass give the five filtered
// moments, and each pixel forms S and dL/d{mu_x, E[x^2], E[xy]}.  Backward:
// those three maps are filtered the same way (the window is symmetric, so
// the adjoint of the correlation is the same correlation) and combined with
// x and y into dL/dR = M dL/dx.  One flat grid over the (view, channel,
// tile) slots of all views; every thread finishes two pixels of its tile.
// Per-tile sums are reduced per view in a fixed order.
#include <cmath>

#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr int kNT = 256;
constexpr int kTX = 32, kTY = 16;                     // output tile (two rows per thread)
constexpr int kR = 5;                                 // window radius
constexpr int kHX = kTX + 2 * kR, kHY = kTY + 2 * kR; // tile with halo
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Taps {
    float g[2 * kR + 1];
};

__host__ __device__ inline int tiles_of(int W, int H) { return ((W + kTX - 1) / kTX) * ((H + kTY - 1) / kTY); }

__device__ __forceinline__ float block_sum(float v, float* s) {
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

// Tile, channel and view of this workgroup (slot = its index among the
// view's 3 * tiles slots); false past the last view.
struct SsimTile {
    int v, ch, x0, y0, W, H, slot;
    int64_t HW, off;
};

__device__ __forceinline__ bool ssim_tile(const sr_camera* cams, int V, SsimTile& t) {
    int b = (int)blockIdx.x, v = 0;
    for (; v < V; ++v) {
        const int ns = 3 * tiles_of(cams[v].width, cams[v].height);
        if (b < ns) break;
        b -= ns;
    }
    if (v >= V) return false;
    t.v = v;
    const sr_camera& c = cams[t.v];
    t.W = c.width;
    t.H = c.height;
    const int nt = tiles_of(t.W, t.H);
    t.ch = b / nt;
    const int tile = b - t.ch * nt;
    const int ntx = (t.W + kTX - 1) / kTX;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    t.x0 = tx * kTX;
    t.y0 = ty * kTY;
    t.HW = (int64_t)t.W * t.H;
    t.off = c.pix_offset;
    t.slot = b;
    return true;
}

// Masked inputs of the tile and its halo (zero outside the image).
__device__ __forceinline__ void load_xy(const SsimTile& t, const float* __restrict__ C, const float* __restrict__ I,
                                        const uint8_t* __restrict__ M, float (&sx)[kHY][kHX],
                                        float (&sy)[kHY][kHX]) {
    for (int k = threadIdx.x; k < kHX * kHY; k += kNT) {
        const int ly = k / kHX, lx = k - ly * kHX;
        const int i = t.x0 - kR + lx, j = t.y0 - kR + ly;
        float xv = 0.f, yv = 0.f;
        if (i >= 0 && i < t.W && j >= 0 && j < t.H) {
            const int64_t p = (int64_t)j * t.W + i;
            const float m = M[p] ? 1.0f : 0.0f;
            xv = m * C[p];
            yv = m * I[p];
        }
        sx[ly][lx] = xv;
        sy[ly][lx] = yv;
    }
}

__global__ void __launch_bounds__(kNT)
k_ssim_fwd(const sr_camera* __restrict__ cams, int V, const float* __restrict__ color,
           const float* __restrict__ target, const uint8_t* __restrict__ mask, Taps taps, float w_s, int nslot,
           int64_t P3, float* __restrict__ partial, float* __restrict__ gmaps) {
#pragma clang fp contract(off)
    __shared__ float sx[kHY][kHX], sy[kHY][kHX];
    __shared__ float sh[5][kHY][kTX];
    __shared__ float s_red[kNT];
    SsimTile t;
    if (!ssim_tile(cams, V, t)) return;               // uniform: the whole block leaves
    const int64_t base = 3 * t.off + t.ch * t.HW;     // this channel of this view in [3P] arrays
    load_xy(t, color + base, target + base, mask + t.off, sx, sy);
    __syncthreads();
    for (int k = threadIdx.x; k < kHY * kTX; k += kNT) {
        const int ly = k / kTX, lx = k - ly * kTX;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int d = 0; d <= 2 * kR; ++d) {
            const float g = taps.g[d], xv = sx[ly][lx + d], yv = sy[ly][lx + d];
            a0 = __builtin_fmaf(g, xv, a0);
            a1 = __builtin_fmaf(g, yv, a1);
            a2 = __builtin_fmaf(g, (xv * xv), a2);
            a3 = __builtin_fmaf(g, (yv * yv), a3);
            a4 = __builtin_fmaf(g, (xv * yv), a4);
        }
        sh[0][ly][lx] = a0; sh[1][ly][lx] = a1; sh[2][ly][lx] = a2; sh[3][ly][lx] = a3; sh[4][ly][lx] = a4;
    }
    __syncthreads();
    const int lx = (int)threadIdx.x % kTX;
    float ssum = 0.f, se = 0.f;
#pragma unroll
    for (int half = 0; half < kTY * kTX / kNT; ++half) {
      const int ly = (int)threadIdx.x / kTX + half * (kNT / kTX);
      const int i = t.x0 + lx, j = t.y0 + ly;
      if (i < t.W && j < t.H) {
        float mx = 0.f, my = 0.f, ex2 = 0.f, ey2 = 0.f, exy = 0.f;
#pragma unroll
        for (int d = 0; d <= 2 * kR; ++d) {
            const float g = taps.g[d];
            mx = __builtin_fmaf(g, sh[0][ly + d][lx], mx);
            my = __builtin_fmaf(g, sh[1][ly + d][lx], my);
            ex2 = __builtin_fmaf(g, sh[2][ly + d][lx], ex2);
            ey2 = __builtin_fmaf(g, sh[3][ly + d][lx], ey2);
            exy = __builtin_fmaf(g, sh[4][ly + d][lx], exy);
        }
        const float vx = ex2 - mx * mx, vy = ey2 - my * my, cxy = exy - mx * my;
        const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = (vx + vy) + kC2;
        const float S = (A1 * A2) / (B1 * B2);
        ssum += S;
        const float xv = sx[ly + kR][lx + kR], yv = sy[ly + kR][lx + kR];
        se += (xv - yv) * (xv - yv);
        if (gmaps) {
            // dL/dS = -w_s / (3 H W V); chain through A1, A2, B1, B2
            const float dS = -w_s / (3.0f * (float)t.HW * (float)V);
            const float d_mx = (((S / A1) * (2.0f * my) - (S / A2) * (2.0f * my)) - (S / B1) * (2.0f * mx)) +
                               (S / B2) * (2.0f * mx);
            const float d_ex2 = -S / B2;
            const float d_exy = 2.0f * (S / A2);
            const int64_t p = base + (int64_t)j * t.W + i;
            gmaps[p] = dS * d_mx;
            gmaps[P3 + p] = dS * d_ex2;
            gmaps[2 * P3 + p] = dS * d_exy;
        }
      }
    }
    ssum = block_sum(ssum, s_red);
    se = block_sum(se, s_red);
    if (threadIdx.x == 0) {
        partial[2 * ((size_t)t.v * nslot + t.slot)] = ssum;
        partial[2 * ((size_t)t.v * nslot + t.slot) + 1] = se;
    }
}

// dL/dx = G*g1 + 2 x G*g2 + y G*g3; dL/dR += M dL/dx
__global__ void __launch_bounds__(kNT)
k_ssim_bwd(const sr_camera* __restrict__ cams, int V, const float* __restrict__ color,
           const float* __restrict__ target,
           const uint8_t* __restrict__ mask, Taps taps, int64_t P3, const float* __restrict__ gmaps,
           float* __restrict__ dL_dcolor) {
#pragma clang fp contract(off)
    __shared__ float sg[3][kHY][kHX];
    __shared__ float sh[3][kHY][kTX];
    SsimTile t;
    if (!ssim_tile(cams, V, t)) return;
    const int64_t base = 3 * t.off + t.ch * t.HW;
    for (int k = threadIdx.x; k < kHX * kHY; k += kNT) {
        const int ly = k / kHX, lx = k - ly * kHX;
        const int i = t.x0 - kR + lx, j = t.y0 - kR + ly;
        float g0 = 0.f, g1 = 0.f, g2 = 0.f;
        if (i >= 0 && i < t.W && j >= 0 && j < t.H) {
            const int64_t p = base + (int64_t)j * t.W + i;
            g0 = gmaps[p];
            g1 = gmaps[P3 + p];
            g2 = gmaps[2 * P3 + p];
        }
        sg[0][ly][lx] = g0; sg[1][ly][lx] = g1; sg[2][ly][lx] = g2;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kHY * kTX; k += kNT) {
        const int ly = k / kTX, lx = k - ly * kTX;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int d = 0; d <= 2 * kR; ++d) {
            const float g = taps.g[d];
            a0 = __builtin_fmaf(g, sg[0][ly][lx + d], a0);
            a1 = __builtin_fmaf(g, sg[1][ly][lx + d], a1);
            a2 = __builtin_fmaf(g, sg[2][ly][lx + d], a2);
        }
        sh[0][ly][lx] = a0; sh[1][ly][lx] = a1; sh[2][ly][lx] = a2;
    }
    __syncthreads();
    const int lx = (int)threadIdx.x % kTX;
#pragma unroll
    for (int half = 0; half < kTY * kTX / kNT; ++half) {
      const int ly = (int)threadIdx.x / kTX + half * (kNT / kTX);
      const int i = t.x0 + lx, j = t.y0 + ly;
      if (i < t.W && j < t.H) {
        float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
        for (int d = 0; d <= 2 * kR; ++d) {
            const float g = taps.g[d];
            f0 = __builtin_fmaf(g, sh[0][ly + d][lx], f0);
            f1 = __builtin_fmaf(g, sh[1][ly + d][lx], f1);
            f2 = __builtin_fmaf(g, sh[2][ly + d][lx], f2);
        }
        const int64_t q = (int64_t)j * t.W + i;
        if (mask[t.off + q]) {
            const float xv = color[base + q], yv = target[base + q];
            const float dx = (f0 + 2.0f * xv * f1) + yv * f2;
            dL_dcolor[base + q] += dx;
        }
      }
    }
}

// out[v] = SSIM_v, out[V+v] = PSNR_v; out[2V] = (1/V) sum_v w_s (1 - SSIM_v)
__global__ void __launch_bounds__(kNT)
k_ssim_final(const sr_camera* __restrict__ cams, int V, int nslot, const float* __restrict__ partial, float w_s,
             float* __restrict__ out) {
    __shared__ float s[kNT];
    for (int v = 0; v < V; ++v) {
        const int ns = 3 * tiles_of(cams[v].width, cams[v].height);
        float a = 0.f, b = 0.f;
        for (int i = threadIdx.x; i < ns; i += kNT) {
            a += partial[2 * ((size_t)v * nslot + i)];
            b += partial[2 * ((size_t)v * nslot + i) + 1];
        }
        a = block_sum(a, s);
        b = block_sum(b, s);
        if (threadIdx.x == 0) {
            const float n = 3.0f * (float)cams[v].width * (float)cams[v].height;
            out[v] = a / n;
            out[V + v] = -10.0f * log10f(b / n);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int v = 0; v < V; ++v) t += w_s * (1.0f - out[v]);
        out[2 * V] = t / (float)V;
    }
}

Taps make_taps() {
    Taps t;
    double g[2 * kR + 1], sum = 0.0;
    for (int k = 0; k <= 2 * kR; ++k) {
        const double d = (double)(k - kR);
        g[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k <= 2 * kR; ++k) t.g[k] = (float)(g[k] / sum);
    return t;
}

}  // namespace

int ssim_slots(int W, int H) { return 3 * tiles_of(W, H); }

size_t ssim_workspace_bytes(int V, int max_slots, int64_t P, bool with_grad) {
    size_t b = (size_t)V * (size_t)max_slots * 2 * sizeof(float);
    b = (b + 255) & ~size_t(255);
    if (with_grad) b += (size_t)3 * 3 * (size_t)P * sizeof(float);
    return b;
}

hipError_t launch_ssim(int V, int max_slots, int total_slots, int64_t P, const sr_camera* cams, const float* color,
                       const float* target, const uint8_t* mask, float w_s, void* ws, float* out,
                       float* dL_dcolor, hipStream_t s) {
    if (V == 0 || max_slots == 0) return hipSuccess;
    const Taps taps = make_taps();
    float* partial = (float*)ws;
    size_t pb = (size_t)V * (size_t)max_slots * 2 * sizeof(float);
    pb = (pb + 255) & ~size_t(255);
    float* gmaps = dL_dcolor ? (float*)((char*)ws + pb) : nullptr;
    const int64_t P3 = 3 * P;
    hipLaunchKernelGGL(k_ssim_fwd, dim3(total_slots), dim3(kNT), 0, s, cams, V, color, target, mask, taps, w_s,
                       max_slots, P3, partial, gmaps);
    if (dL_dcolor)
        hipLaunchKernelGGL(k_ssim_bwd, dim3(total_slots), dim3(kNT), 0, s, cams, V, color, target, mask, taps, P3,
                           (const float*)gmaps, dL_dcolor);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(kNT), 0, s, cams, V, max_slots, (const float*)partial, w_s, out);
    return hipGetLastError();
}

}  // namespace sr
