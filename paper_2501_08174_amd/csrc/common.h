// Internal device helpers shared by the surfel rasterizer kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "surfelrast.h"

namespace sr {

constexpr int kGeomF4 = SR_GEOM_STRIDE / 4;   // float4 per geometry record
constexpr int kAppF4 = SR_APP_STRIDE / 4;     // float4 per appearance record
constexpr int kNumGrad = 21;                  // gradient floats per record

// Constants of the compositing rule, passed by value to the raster kernels.
struct RasterConsts {
    float alpha_min;
    float alpha_max;
    float t_min;
    uint32_t flags;
    // the context's device status word (NULL: none); while it is set the
    // instance lists are truncated and the compositing kernels compute nothing
    const uint32_t* status;
};

// The status word's verdict, read once per workgroup (uniform).
__device__ __forceinline__ bool status_failed(const RasterConsts& rc) {
    return rc.status != nullptr && *rc.status != 0u;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Neighbouring tiles read mostly the same surfel records, so give every XCD a
// contiguous run of tiles: block b of round r = b / 8 on XCD x = b % 8 takes
// tile x * (G / 8) + r.  The last G % 8 blocks keep their own id (bijection).
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int full = G >> 3;
    if (b >= (full << 3)) return b;
    return (b & 7) * full + (b >> 3);
}

// View that owns a global tile id (views are stored in tile order).
__device__ __forceinline__ int view_of_tile(const sr_camera* __restrict__ cams, int V, int tile) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int view_of_group(const sr_camera* __restrict__ cams, int V, int group) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cams[mid].group_offset <= group) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sorted instance values: surfel id in the low SR_INST_ID_BITS bits, the
// surfel's tile rectangle clipped to the group (2-bit tile coordinates
// x_lo, x_hi, y_lo, y_hi inside the group) above.
constexpr uint32_t kInstIdMask = (1u << SR_INST_ID_BITS) - 1u;
__device__ __forceinline__ bool inst_covers(uint32_t v, int sx, int sy) {
    const uint32_t sub = v >> SR_INST_ID_BITS;
    return (int)(sub & 3u) <= sx && sx <= (int)((sub >> 2) & 3u) && (int)((sub >> 4) & 3u) <= sy &&
           sy <= (int)((sub >> 6) & 3u);
}

// ---------------------------------------------------------------------------
// Wavefront (64 lanes) reductions with DPP row operations.  Results land in
// lane 63.  Must be called with all 64 lanes active.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Wave-wide sums of N per-lane values (N = 8 or 16) by transposition: at
// every step the values of two registers are exchanged between the two halves
// of the lanes being combined, so each step halves both the number of
// registers and the number of lanes that share a value.  Halves of the wave
// (lanes l, l^32) and pairs of rows (l, l^16) are combined with the gfx950
// permlane swaps, lanes l, l^1 and l, l^2 with DPP quad permutations, the
// remaining lanes l, l^4, l^8 with row rotations.  On return every lane holds
// the wave total of component wave_tsum_comp<N>(lane).
template <int N>
__device__ __forceinline__ int wave_tsum_comp(int lane) {
    const int r = lane >> 4;
    const int pr = ((r & 1) << 1) | (r >> 1);   // row 0,1,2,3 -> 0,2,1,3
    const int p = lane & 1;
    if (N == 16) return 8 * ((lane >> 1) & 1) + 4 * p + pr;
    return 4 * p + pr;
}

template <int N>
__device__ __forceinline__ float wave_tsum(const float* v) {
    static_assert(N == 8 || N == 16, "8 or 16 components");
    float s[N / 2];
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * j]), __float_as_uint(v[2 * j + 1]),
                                                        false, false);
        s[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float t[N / 4];
#pragma unroll
    for (int m = 0; m < N / 4; ++m) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[2 * m]), __float_as_uint(s[2 * m + 1]),
                                                        false, false);
        t[m] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool odd = (__lane_id() & 1) != 0;
    float u[N / 8];
#pragma unroll
    for (int n = 0; n < N / 8; ++n) {
        const float keep = odd ? t[2 * n + 1] : t[2 * n];
        const float send = odd ? t[2 * n] : t[2 * n + 1];
        u[n] = keep + dpp_f<0xB1, 0xF>(send);   // quad_perm [1,0,3,2]
    }
    float w;
    if (N == 16) {
        const bool b1 = (__lane_id() & 2) != 0;
        const float keep = b1 ? u[1] : u[0];
        const float send = b1 ? u[0] : u[1];
        w = keep + dpp_f<0x4E, 0xF>(send);      // quad_perm [2,3,0,1]
    } else {
        w = u[0] + dpp_f<0x4E, 0xF>(u[0]);
    }
    w += dpp_f<0x124, 0xF>(w);                  // row_ror:4
    w += dpp_f<0x128, 0xF>(w);                  // row_ror:8
    return w;
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Wave maxima of two non-negative floats, compared as their bit patterns
// (which order like the values): the halves of the wave exchange a and b, the
// row pairs exchange again, then each row reduces with DPP.  On return lanes
// 0..31 hold the bits of max(a) over the wave and lanes 32..63 those of max(b).
__device__ __forceinline__ uint32_t wave_max2_bits(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    uint32_t m = r[0] > r[1] ? r[0] : r[1];
    const auto q = __builtin_amdgcn_permlane16_swap(m, m, false, false);
    m = q[0] > q[1] ? q[0] : q[1];
    uint32_t d;
    d = dpp_u<0xB1>(m); m = m > d ? m : d;    // quad_perm [1,0,3,2]
    d = dpp_u<0x4E>(m); m = m > d ? m : d;    // quad_perm [2,3,0,1]
    d = dpp_u<0x141>(m); m = m > d ? m : d;   // row_half_mirror
    d = dpp_u<0x140>(m); m = m > d ? m : d;   // row_mirror
    return m;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// Evaluation of one (pixel, surfel) pair.  Shared verbatim by the forward,
// backward and pruning kernels so that they take identical decisions: every
// operation is written explicitly and contraction is disabled.
//
// Geometry record (16 floats), for pixel centre x and dx = x - c:
//   w = A dx + B dy + C  (w ~ (u, v, 1): inverse of the splat homography),
//   c = projected centre, o = opacity, m3 = (a_u.z, a_v.z, p_z) so that the
//   surface depth is m3 . (u, v, 1), L = ln(o / alpha_min).
//   [A0 A1 A2 B0 | B1 B2 C0 C1 | C2 cx cy o | m30 m31 m32 L]
// An entry passes the alpha cutoff when min(rho_s/2, rho_f) <= L with
// rho_s = u^2 + v^2 and rho_f = |x - c|^2, i.e. o exp(-rho) >= alpha_min.
// ---------------------------------------------------------------------------
struct PairEval {
    float dx, dy, w0, w1, w2, rho_f;
    bool pass, s_ok;
    float r, u, v, rho, G, a, z;   // r = 1/w2
    bool surf, clamped;
};

// Stage 1: the cutoff test (no division, no exponential).
__device__ __forceinline__ void eval_test(const float4& g0, const float4& g1, const float4& g2,
                                          const float4& g3, float px, float py, PairEval& e) {
#pragma clang fp contract(off)
    e.dx = px - g2.y;
    e.dy = py - g2.z;
    e.w0 = __builtin_fmaf(g0.x, e.dx, __builtin_fmaf(g0.w, e.dy, g1.z));
    e.w1 = __builtin_fmaf(g0.y, e.dx, __builtin_fmaf(g1.x, e.dy, g1.w));
    e.w2 = __builtin_fmaf(g0.z, e.dx, __builtin_fmaf(g1.y, e.dy, g2.x));
    const float L = g3.w;
    e.rho_f = __builtin_fmaf(e.dx, e.dx, e.dy * e.dy);
    const float q = __builtin_fmaf(e.w0, e.w0, e.w1 * e.w1);
    const float w22 = e.w2 * e.w2;
    e.s_ok = (q <= (2.0f * L) * w22) && (e.w2 != 0.0f);
    e.pass = e.s_ok || (e.rho_f <= L);
}

// Stage 2: intersection, Gaussian value, alpha and depth of a passing pair.
__device__ __forceinline__ void eval_finish(const float4& g2, const float4& g3, float alpha_max, PairEval& e) {
#pragma clang fp contract(off)
    e.r = __builtin_amdgcn_rcpf(e.w2);
    e.u = e.w0 * e.r;
    e.v = e.w1 * e.r;
    const float rho_s = 0.5f * __builtin_fmaf(e.u, e.u, e.v * e.v);
    e.surf = e.s_ok && (rho_s <= e.rho_f);
    e.rho = e.surf ? rho_s : e.rho_f;
    // exp(-rho) = 2^(-rho log2 e)
    e.G = __builtin_amdgcn_exp2f(-1.4426950408889634f * e.rho);
    const float oG = g2.w * e.G;
    e.clamped = oG > alpha_max;
    // min(oG, alpha_max) as the median of (oG, 0, alpha_max): oG >= 0, and
    // one instruction where the select needs the bound in a vector register
    e.a = __builtin_amdgcn_fmed3f(oG, 0.0f, alpha_max);
    e.z = e.surf ? __builtin_fmaf(g3.x, e.u, __builtin_fmaf(g3.y, e.v, g3.z)) : g3.z;
}

// Per-pixel terms of the masked losses (Eq. 1 and the L1 part of Eq. 2) and
// their gradients for L = (1/V) sum_v (w_c L1_v + gamma L_b,v); shared by the
// loss kernel and the fused training step so both round identically.
__device__ __forceinline__ void pixel_loss_grad(uint8_t mask, float A, const float* C, const float* I, float gamma,
                                                float w_c, float HW, float V, float& lb, float& l1, float& gA,
                                                float* gC) {
#pragma clang fp contract(off)
    const float ga = gamma / (HW * V);
    const float gc = w_c / (3.0f * HW * V);
    const float m = mask ? 1.0f : 0.0f;
    lb += A * (1.0f - m);
    gA = ga * (1.0f - m);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float d = m * C[ch] - m * I[ch];
        l1 += fabsf(d);
        gC[ch] = d > 0.f ? gc * m : (d < 0.f ? -gc * m : 0.f);
    }
}

}  // namespace sr
