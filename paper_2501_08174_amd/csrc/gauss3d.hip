// Occlusion-aware pruning statistics for 3D Gaussians (Appendix B: the
// pruning of Section 4.3 applied to 3DGS).  The 3D Gaussians are splatted as
// 2D Gaussians (EWA: Sigma_2 = J R_v Sigma R_v^T J^T + 0.3 I with the
// clamped-field-of-view Jacobian of 3DGS), binned and sorted with the same
// instance machinery as the surfels, and composited front to back with the
// surfel path's cutoff, clamp and termination rules; only the occlusion
// statistics are produced.
//
// Projection and binning run in float64 in a fixed operation order (no
// contraction, IEEE division and square root, the logarithm rounded up to the
// 2^-16 grid), so that the conservative pixel rectangles, tile counts and
// depth keys are bit-identical with the float64 oracle.
#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr double kGrid3 = 65536.0;
constexpr double kDilation = 0.3;
constexpr double kFovClamp = 1.3;

__global__ void k_zero_flags(uint8_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ double rowdot3(const double* r, double a0, double a1, double a2) {
#pragma clang fp contract(off)
    return (r[0] * a0 + r[1] * a1) + r[2] * a2;
}

// One thread per (Gaussian g, view v), t = g * V + v.
__global__ void __launch_bounds__(256)
k_preprocess3d(int N, const float* __restrict__ means, const float* __restrict__ scales,
               const float* __restrict__ quats, const float* __restrict__ opac, float alpha_min, int tile_w,
               int tile_h, int V, const sr_camera* __restrict__ cams, float4* __restrict__ geom3,
               ushort4* __restrict__ rect, uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ depth_key,
               uint8_t* __restrict__ in_frustum) {
#pragma clang fp contract(off)
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint64_t)N * (uint64_t)V) return;
    const int g = (int)(t / (uint64_t)V);
    const int v = (int)(t - (uint64_t)g * (uint64_t)V);
    const size_t r = (size_t)v * N + g;
    const sr_camera& cam = cams[v];
    double R[9], tv[3];
    for (int i = 0; i < 3; ++i) {
        R[3 * i + 0] = (double)cam.viewmat[4 * i + 0];
        R[3 * i + 1] = (double)cam.viewmat[4 * i + 1];
        R[3 * i + 2] = (double)cam.viewmat[4 * i + 2];
        tv[i] = (double)cam.viewmat[4 * i + 3];
    }
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy, znear = cam.znear;
    const double mu[3] = {(double)means[3 * g], (double)means[3 * g + 1], (double)means[3 * g + 2]};
    const double s[3] = {(double)scales[3 * g], (double)scales[3 * g + 1], (double)scales[3 * g + 2]};
    const float o32 = opac[g];
    const double o = o32;
    double w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
    const double nrm = sqrt(((w * w + x * x) + y * y) + z * z);
    w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
    // columns of R(q)
    const double c0[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
    const double c1[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
    const double c2[3] = {2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)};
    // columns of W = R_v R S, and the camera-space centre
    double W0[3], W1[3], W2[3], p[3];
    for (int i = 0; i < 3; ++i) {
        W0[i] = rowdot3(&R[3 * i], c0[0], c0[1], c0[2]) * s[0];
        W1[i] = rowdot3(&R[3 * i], c1[0], c1[1], c1[2]) * s[1];
        W2[i] = rowdot3(&R[3 * i], c2[0], c2[1], c2[2]) * s[2];
        p[i] = rowdot3(&R[3 * i], mu[0], mu[1], mu[2]) + tv[i];
    }
    const double px = p[0], py = p[1], pz = p[2];
    const double limx = kFovClamp * ((double)cam.width / (2.0 * fx));
    const double limy = kFovClamp * ((double)cam.height / (2.0 * fy));
    const double tx = fmin(limx, fmax(-limx, px / pz)) * pz;
    const double ty = fmin(limy, fmax(-limy, py / pz)) * pz;
    const double j00 = fx / pz, j02 = -(fx * tx) / (pz * pz);
    const double j11 = fy / pz, j12 = -(fy * ty) / (pz * pz);
    // rows of U = J W
    const double* Wc[3] = {W0, W1, W2};
    double u0[3], u1[3];
    for (int k = 0; k < 3; ++k) {
        u0[k] = j00 * Wc[k][0] + j02 * Wc[k][2];
        u1[k] = j11 * Wc[k][1] + j12 * Wc[k][2];
    }
    const double ca = ((u0[0] * u0[0] + u0[1] * u0[1]) + u0[2] * u0[2]) + kDilation;
    const double cb = (u0[0] * u1[0] + u0[1] * u1[1]) + u0[2] * u1[2];
    const double cc = ((u1[0] * u1[0] + u1[1] * u1[1]) + u1[2] * u1[2]) + kDilation;
    const double det = ca * cc - cb * cb;
    const double L = log(o / (double)alpha_min);
    const double r2 = ceil((2.0 * L) * kGrid3) / kGrid3;
    const double ccx = (fx * px) / pz + cx, ccy = (fy * py) / pz + cy;
    const double ex = sqrt(r2 * ca), ey = sqrt(r2 * cc);
    const double flo = fmax(ceil((ccx - ex) - 0.5), 0.0), fhi = fmin(floor((ccx + ex) - 0.5), cam.width - 1.0);
    const double glo = fmax(ceil((ccy - ey) - 0.5), 0.0), ghi = fmin(floor((ccy + ey) - 0.5), cam.height - 1.0);
    // numpy-style NaN semantics: any NaN empties the rectangle
    const bool nan = isnan(ccx) || isnan(ccy) || isnan(ex) || isnan(ey);
    const bool culled = (pz <= znear) || (o32 < alpha_min) || !(det > 0.0) || nan || !(flo <= fhi) ||
                        !(glo <= ghi);
    if (culled) {
        tiles_touched[r] = 0u;
        depth_key[r] = 0xFFFFFFFFu;
        rect[r] = make_ushort4(0, 0, 0, 0);
        return;
    }
    if (in_frustum) in_frustum[g] = 1;
    const int ilo = (int)flo, ihi = (int)fhi, jlo = (int)glo, jhi = (int)ghi;
    const int txlo = ilo / tile_w, txhi = ihi / tile_w, tylo = jlo / tile_h, tyhi = jhi / tile_h;
    tiles_touched[r] = (uint32_t)((txhi - txlo + 1) * (tyhi - tylo + 1));
    depth_key[r] = __float_as_uint((float)pz);
    rect[r] = make_ushort4((unsigned short)ilo, (unsigned short)ihi, (unsigned short)jlo, (unsigned short)jhi);
    geom3[2 * r + 0] = make_float4((float)(cc / det), (float)(-cb / det), (float)(ca / det), o32);
    geom3[2 * r + 1] = make_float4((float)ccx, (float)ccy, (float)L, 0.0f);
}

// Bits of the waves that the cutoff ellipse q = a dx^2 + 2 b dx dy + c dy^2
// <= 2 L of one record can reach.  Every wave covers an 8x8 block of the tile
// (wave w: block column w % (TW / 8), block row w / (TW / 8)); float64 with a
// relative slack tau on 2 L and a 1e-3 pixel margin (an entry is skipped
// only where the exact test fails by a margin).  For fixed dx the ellipse is
// the interval of dy between the roots of c dy^2 + 2 b dx dy + a dx^2 - 2 L;
// its lower end is convex and its upper end concave in dx, so their extremes
// over a block's columns sit at the lowest / highest point of the ellipse
// clamped to those columns.
constexpr int kWaveBlock3d = 8;

template <int TW, int NW>
__device__ __forceinline__ uint32_t band_bits3d(const float4& c0, const float4& c1, int tx0, int ty0) {
    constexpr int WB = kWaveBlock3d;
    static_assert(TW % WB == 0 && NW % (TW / WB) == 0, "waves cover whole 8x8 blocks of the tile");
    constexpr int BX = TW / WB, BY = NW / BX;
    constexpr double tau = 1e-3, mg = 1e-3;
    const double a = c0.x, b = c0.y, c = c0.z, cx = c1.x, cy = c1.y;
    const double r2 = 2.0 * (double)c1.z * (1.0 + tau);
    const double det = a * c - b * b;
    if (!(a > 0.0 && c > 0.0 && det > 0.0)) return (1u << NW) - 1u;     // not an ellipse: keep
    const double hx = sqrt(r2 * c / det);                  // the ellipse's half width
    const double hy = sqrt(r2 * a / det);                  // lowest / highest points at dy = -+hy
    uint32_t bits = 0u;
#pragma unroll
    for (int bx = 0; bx < BX; ++bx) {
        const double X0 = (tx0 + bx * WB + 0.5) - cx - mg, X1 = (tx0 + bx * WB + WB - 0.5) - cx + mg;
        const double xa = fmax(X0, -hx), xb = fmin(X1, hx);
        if (xa > xb) continue;
        const double xbot = fmin(fmax(b * hy / a, xa), xb), xtop = fmin(fmax(-b * hy / a, xa), xb);
        const double ylo = (-b * xbot - sqrt(fmax(r2 * c - det * xbot * xbot, 0.0))) / c;
        const double yhi = (-b * xtop + sqrt(fmax(r2 * c - det * xtop * xtop, 0.0))) / c;
#pragma unroll
        for (int by = 0; by < BY; ++by) {
            const double Y0 = (ty0 + by * WB + 0.5) - cy - mg, Y1 = (ty0 + by * WB + WB - 0.5) - cy + mg;
            if (ylo <= Y1 && yhi >= Y0) bits |= 1u << (by * BX + bx);
        }
    }
    return bits;
}

// Front to back over a tile's list; every thread owns one pixel; only the
// occlusion statistics (hits, max alpha, max weight) are written.  Each
// wave walks only the entries whose ellipse reaches its block.
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_prune3d(const sr_camera* __restrict__ cams, int V, int N, const float4* __restrict__ geom3,
          const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges, RasterConsts rc,
          uint32_t* __restrict__ hits, float* __restrict__ max_alpha, float* __restrict__ max_weight) {
#pragma clang fp contract(off)
    constexpr int NT = TW * TH;
    __shared__ float4 sg[2][NT];
    __shared__ uint32_t sid[NT];
    __shared__ uint32_t sst[3][NT];   // per-batch hits, max alpha, max weight over the waves
    if (status_failed(rc)) return;    // truncated lists: no statistics
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = view_of_tile(cams, V, tile);
    const sr_camera& c = cams[v];
    const int local = tile - c.tile_offset;
    const int ty = local / c.tiles_x, tx = local - ty * c.tiles_x;
    // wave w covers the 8x8 block (w % (TW / 8), w / (TW / 8)) of the tile
    constexpr int WB = kWaveBlock3d;
    const int wt = (int)threadIdx.x >> 6, lt = (int)threadIdx.x & 63;
    const int ix = tx * TW + (wt % (TW / WB)) * WB + (lt % WB), iy = ty * TH + (wt / (TW / WB)) * WB + lt / WB;
    const int wv = (int)__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6;
    const float px = (float)ix + 0.5f, py = (float)iy + 0.5f;
    const uint2 rg = ranges[tile];
    const uint32_t start = rg.x, n = rg.y - rg.x;
    const int lane = __lane_id();
    float T = 1.0f;
    bool done = !(ix < c.width && iy < c.height);
    for (uint32_t base = 0; base < n; base += NT) {
        if (__syncthreads_and(done)) break;
        const uint32_t j = base + threadIdx.x;
        if (j < n) {
            // the group's run holds entries for the other tiles of the group too
            const uint32_t gv = vals[start + j];
            const uint32_t gg = gv & kInstIdMask;
            if (inst_covers(gv, tx % SR_TILE_GROUP, ty % SR_TILE_GROUP)) {
                const size_t r = (size_t)v * N + gg;
                const float4 c0 = geom3[2 * r], c1 = geom3[2 * r + 1];
                sg[0][threadIdx.x] = c0;
                // the wave bits take the record's unused last slot
                sg[1][threadIdx.x] = make_float4(c1.x, c1.y, c1.z,
                                                 __uint_as_float(band_bits3d<TW, NT / 64>(c0, c1, tx * TW, ty * TH)));
            } else {
                sg[1][threadIdx.x].w = 0.f;
            }
            sid[threadIdx.x] = gg;
            sst[0][threadIdx.x] = 0u;
            sst[1][threadIdx.x] = 0u;
            sst[2][threadIdx.x] = 0u;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, n - base);
        bool wave_done = __ballot(!done) == 0ull;
        for (int cr = 0; cr * 64 < cnt && !wave_done; ++cr) {
          const int kk = cr * 64 + lane;
          uint64_t live = __ballot(kk < cnt && ((__float_as_uint(sg[1][kk < cnt ? kk : 0].w) >> wv) & 1u));
          while (live != 0ull) {
            const int k = cr * 64 + (int)__builtin_ctzll(live);
            live &= live - 1ull;
            const float4 a0 = sg[0][k], a1 = sg[1][k];
            const float dx = px - a1.x, dy = py - a1.y;
            const float q = (a0.x * dx * dx + 2.0f * a0.y * dx * dy) + a0.z * dy * dy;
            bool blend = !done && (0.5f * q <= a1.z);
            if (__ballot(blend) == 0ull) continue;
            const float G = __builtin_amdgcn_exp2f(-0.72134752044448170f * q);   // exp(-q/2)
            const float oG = a0.w * G;
            const float a = oG > rc.alpha_max ? rc.alpha_max : oG;
            const float Tn = T * (1.0f - a);
            if (blend && Tn < rc.t_min) {
                done = true;
                blend = false;
            }
            const float wgt = blend ? a * T : 0.f;
            if (blend) T = Tn;
            const uint64_t bm = __ballot(blend);
            if (bm != 0ull) {
                const uint32_t mx = wave_max2_bits(blend ? a : 0.f, wgt);
                if ((lane & 31) == 0) {
                    if (lane == 0) atomicAdd(&sst[0][k], (uint32_t)__popcll(bm));
                    atomicMax(&sst[lane == 0 ? 1 : 2][k], mx);
                }
            }
            if (__ballot(!done) == 0ull) {
                wave_done = true;
                break;
            }
          }
        }
        // the batch's statistics reach memory once per (tile, entry)
        __syncthreads();
        if ((int)threadIdx.x < cnt && sst[0][threadIdx.x] != 0u) {
            const uint32_t g = sid[threadIdx.x];
            atomicAdd(&hits[g], sst[0][threadIdx.x]);
            atomicMax((uint32_t*)&max_alpha[g], sst[1][threadIdx.x]);
            atomicMax((uint32_t*)&max_weight[g], sst[2][threadIdx.x]);
        }
    }
}

}  // namespace

hipError_t launch_preprocess3d(const sr_config& cfg, int N, const float* means, const float* scales,
                               const float* quats, const float* opac, int V, const sr_camera* cams_dev,
                               float* geom3, uint16_t* rect, uint32_t* tiles_touched, uint32_t* depth_key,
                               uint8_t* in_frustum, hipStream_t s) {
    if (N == 0) return hipSuccess;
    if (in_frustum && !(cfg.flags & SR_FLAG_ACCUMULATE))
        hipLaunchKernelGGL(k_zero_flags, dim3((N + 255) / 256), dim3(256), 0, s, in_frustum, N);
    const uint64_t threads = (uint64_t)N * (uint64_t)V;
    if (threads == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_preprocess3d, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, N, means, scales,
                       quats, opac, cfg.alpha_min, cfg.tile_w, cfg.tile_h, V, cams_dev, (float4*)geom3,
                       (ushort4*)rect, tiles_touched, depth_key, in_frustum);
    return hipGetLastError();
}

hipError_t launch_prune3d(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                          const float* geom3, const uint32_t* vals, const uint32_t* ranges, uint32_t* hits,
                          float* max_alpha, float* max_weight, const uint32_t* status, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    const RasterConsts rc{cfg.alpha_min, cfg.alpha_max, cfg.t_min, cfg.flags, status};
#define SR_P3(TW, TH)                                                                                          \
    if (cfg.tile_w == TW && cfg.tile_h == TH) {                                                              \
        hipLaunchKernelGGL((k_prune3d<TW, TH>), dim3(total_tiles), dim3(TW * TH), 0, s, cams, V, N,          \
                           (const float4*)geom3, vals, (const uint2*)ranges, rc, hits, max_alpha, max_weight); \
        return hipGetLastError();                                                                            \
    }
    SR_P3(16, 16) SR_P3(16, 8) SR_P3(8, 8) SR_P3(32, 8)
#undef SR_P3
    return hipErrorInvalidValue;
}

}  // namespace sr
