// Projection of surfels into every view of a batch, and its backward.
//
// Section 4.3 of the paper: every Gaussian inside the viewing frustum is
// projected to the image and assigned the pixels it can contribute to; one
// outside is disqualified.  Section 3.1: a surfel carries position, shape
// and appearance, all updated by backpropagation.
//
// The parameters (up to 232 bytes with degree-3 colour) are read from HBM
// once per batch: one thread per surfel loops over the views (large
// batches), or the views of a surfel sit in adjacent lanes.  Culling,
// the pixel rectangle and the depth key are evaluated in float64 in a fixed
// operation order (no contraction, IEEE division and square root) so that
// they are reproducible bit for bit; the records handed to the raster
// kernels are rounded to float32.
#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr double kGrid = 65536.0;   // the cutoff radii are rounded up to 2^-16
// the surfel-loop projection kernel from this many surfels on (three
// workgroups of 256 threads per compute unit)
constexpr int kPreprocessLoopMinSurfels = 3 * 256 * 256;

// Real spherical harmonics up to degree 3 (orthonormal, Condon-Shortley
// phase), l-major, m = -l..l.  Constants: 1/(2 sqrt(pi)), sqrt(3/(4 pi)),
// sqrt(15/(4 pi)), sqrt(5/(16 pi)), sqrt(15/(16 pi)), sqrt(35/(32 pi)),
// sqrt(105/(4 pi)), sqrt(21/(32 pi)), sqrt(7/(16 pi)), sqrt(105/(16 pi)).
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.4886025119029199f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.5462742152960396f;
constexpr float kY3a = 0.5900435899266435f;
constexpr float kY3b = 2.890611442640554f;
constexpr float kY3c = 0.4570457994644658f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.445305721320277f;

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
    Y[0] = kY0;
    if (deg < 1) return;
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (3.0f * zz - 1.0f);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -kY3a * y * (3.0f * xx - yy);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (5.0f * zz - 1.0f);
    Y[12] = kY3d * z * (5.0f * zz - 3.0f);
    Y[13] = -kY3c * x * (5.0f * zz - 1.0f);
    Y[14] = kY3e * z * (xx - yy);
    Y[15] = -kY3a * x * (xx - 3.0f * yy);
}

// Gradient of the polynomial basis above with respect to (x, y, z).
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float* gx, float* gy,
                                              float* gz) {
    gx[0] = gy[0] = gz[0] = 0.0f;
    if (deg < 1) return;
    gx[1] = 0.0f;  gy[1] = -kY1;  gz[1] = 0.0f;
    gx[2] = 0.0f;  gy[2] = 0.0f;  gz[2] = kY1;
    gx[3] = -kY1;  gy[3] = 0.0f;  gz[3] = 0.0f;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx[4] = kY2a * y;          gy[4] = kY2a * x;          gz[4] = 0.0f;
    gx[5] = 0.0f;              gy[5] = -kY2a * z;         gz[5] = -kY2a * y;
    gx[6] = 0.0f;              gy[6] = 0.0f;              gz[6] = 6.0f * kY2b * z;
    gx[7] = -kY2a * z;         gy[7] = 0.0f;              gz[7] = -kY2a * x;
    gx[8] = 2.0f * kY2c * x;   gy[8] = -2.0f * kY2c * y;  gz[8] = 0.0f;
    if (deg < 3) return;
    gx[9] = -6.0f * kY3a * x * y;          gy[9] = -3.0f * kY3a * (xx - yy);     gz[9] = 0.0f;
    gx[10] = kY3b * y * z;                 gy[10] = kY3b * x * z;                gz[10] = kY3b * x * y;
    gx[11] = 0.0f;                         gy[11] = -kY3c * (5.0f * zz - 1.0f);  gz[11] = -10.0f * kY3c * y * z;
    gx[12] = 0.0f;                         gy[12] = 0.0f;                        gz[12] = kY3d * (15.0f * zz - 3.0f);
    gx[13] = -kY3c * (5.0f * zz - 1.0f);   gy[13] = 0.0f;                        gz[13] = -10.0f * kY3c * x * z;
    gx[14] = 2.0f * kY3e * x * z;          gy[14] = -2.0f * kY3e * y * z;        gz[14] = kY3e * (xx - yy);
    gx[15] = -3.0f * kY3a * (xx - yy);     gy[15] = 6.0f * kY3a * x * y;         gz[15] = 0.0f;
}

struct Cam64 {
    double R[9], t[3];
    double fx, fy, cx, cy, znear;
    int W, H, tiles_x;
};

__device__ __forceinline__ void load_cam64(const sr_camera& c, Cam64& k) {
    for (int i = 0; i < 3; ++i) {
        k.R[3 * i + 0] = (double)c.viewmat[4 * i + 0];
        k.R[3 * i + 1] = (double)c.viewmat[4 * i + 1];
        k.R[3 * i + 2] = (double)c.viewmat[4 * i + 2];
        k.t[i] = (double)c.viewmat[4 * i + 3];
    }
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy; k.znear = c.znear;
    k.W = c.width; k.H = c.height; k.tiles_x = c.tiles_x;
}

// ((r0 a0 + r1 a1) + r2 a2), no contraction
__device__ __forceinline__ double rowdot(const double* r, double a0, double a1, double a2) {
#pragma clang fp contract(off)
    return (r[0] * a0 + r[1] * a1) + r[2] * a2;
}

__device__ __forceinline__ double conic_dot(double rs2, const double* a, const double* b) {
#pragma clang fp contract(off)
    return rs2 * (a[0] * b[0] + a[1] * b[1]) - a[2] * b[2];
}

__device__ __forceinline__ double ceil_grid(double x) {
#pragma clang fp contract(off)
    return ceil(x * kGrid) / kGrid;
}

__device__ __forceinline__ void cross3d(const double* a, const double* b, double* o) {
#pragma clang fp contract(off)
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// The per-(view, surfel) outputs of the projection.
struct PreRec {
    float4 geom[4];
    float4 app[2];
    uint32_t rx, ry;          // x_lo | x_hi << 16, y_lo | y_hi << 16: the ushort4 rectangle's bytes
    uint32_t tiles, key;      // tiles = 0: culled (geom, app not written)
};

// Colour of a surfel seen from campos: max(0, sum_k Y_k(d) f_k + 1/2) per
// channel, d the unit direction from the camera centre to the surfel
// (float32; coefficients at f[i * SH_STEP]).
template <int DEG, int SH_STEP>
__device__ __forceinline__ void view_colour(const float* mu32, const float* campos, const float* f, float* rgb) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    float d0 = mu32[0] - campos[0], d1 = mu32[1] - campos[1], d2 = mu32[2] - campos[2];
    const float inv = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    d0 *= inv; d1 *= inv; d2 *= inv;
    float Y[16];
    sh_basis(DEG, d0, d1, d2, Y);
    rgb[0] = rgb[1] = rgb[2] = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        rgb[0] = __builtin_fmaf(Y[k], f[(3 * k + 0) * SH_STEP], rgb[0]);
        rgb[1] = __builtin_fmaf(Y[k], f[(3 * k + 1) * SH_STEP], rgb[1]);
        rgb[2] = __builtin_fmaf(Y[k], f[(3 * k + 2) * SH_STEP], rgb[2]);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = rgb[ch] > 0.0f ? rgb[ch] : 0.0f;
}

// The view-independent terms of a surfel's projection.
struct SurfelTerms {
    double mu[3], su, sv;
    double tu[3], tv[3], nn[3];     // frame: columns of R(q / |q|)
    double L, rs2, rf;              // ln(o / alpha_min), squared cutoff radii, low-pass radius
    float o32;
    bool cull_opac;
};

__device__ __forceinline__ void surfel_terms(int g, const float* __restrict__ means,
                                             const float* __restrict__ scales, const float* __restrict__ quats,
                                             const float* __restrict__ opac, float alpha_min, SurfelTerms& s) {
#pragma clang fp contract(off)
    s.mu[0] = means[3 * g]; s.mu[1] = means[3 * g + 1]; s.mu[2] = means[3 * g + 2];
    s.su = scales[2 * g]; s.sv = scales[2 * g + 1];
    s.o32 = opac[g];
    const double o = s.o32;
    // unit quaternion and the frame (t_u, t_v, n) = columns of R(q)
    double w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
    const double nrm = sqrt(((w * w + x * x) + y * y) + z * z);
    w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
    s.tu[0] = 1.0 - 2.0 * (y * y + z * z); s.tu[1] = 2.0 * (x * y + w * z); s.tu[2] = 2.0 * (x * z - w * y);
    s.tv[0] = 2.0 * (x * y - w * z); s.tv[1] = 1.0 - 2.0 * (x * x + z * z); s.tv[2] = 2.0 * (y * z + w * x);
    s.nn[0] = 2.0 * (x * z + w * y); s.nn[1] = 2.0 * (y * z - w * x); s.nn[2] = 1.0 - 2.0 * (x * x + y * y);
    // cutoff radii: o G >= alpha_min  <=>  rho <= L
    s.L = log(o / (double)alpha_min);
    s.rs2 = ceil_grid(2.0 * s.L);
    s.rf = sqrt(ceil_grid(s.L));
    s.cull_opac = s.o32 < alpha_min;
}

// DEG: SH degree of the colour (0..3), or -1 to skip shading (pruning pass).
// Projects surfel g (its view-independent terms s, its float32 centre mu32
// and colour coefficients shg[i * SH_STEP]) into view v; returns false when
// it is culled.
template <int DEG, int SH_STEP>
__device__ __forceinline__ bool project_view(const SurfelTerms& s, const float* mu32, const float* shg, int v,
                                             int tile_wl, int tile_hl, const sr_camera* __restrict__ cams,
                                             PreRec& out) {
#pragma clang fp contract(off)
    const double* mu = s.mu;
    const double su = s.su, sv = s.sv, L = s.L, rs2 = s.rs2, rf = s.rf;
    const double *tu = s.tu, *tv = s.tv, *nn = s.nn;
    const float o32 = s.o32;
    const bool cull_opac = s.cull_opac;

    Cam64 c;
    load_cam64(cams[v], c);
    double p[3], au[3], av[3], nc[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = rowdot(&c.R[3 * i], mu[0], mu[1], mu[2]) + c.t[i];
        au[i] = su * rowdot(&c.R[3 * i], tu[0], tu[1], tu[2]);
        av[i] = sv * rowdot(&c.R[3 * i], tv[0], tv[1], tv[2]);
        nc[i] = rowdot(&c.R[3 * i], nn[0], nn[1], nn[2]);
    }
    const double dnp = (nc[0] * p[0] + nc[1] * p[1]) + nc[2] * p[2];
    if (dnp > 0.0) { nc[0] = -nc[0]; nc[1] = -nc[1]; nc[2] = -nc[2]; }
    // rows of M = K [a_u a_v p]
    double m1[3], m2[3], m3[3];
    const double* col[3] = {au, av, p};
    for (int j = 0; j < 3; ++j) {
        m1[j] = c.fx * col[j][0] + c.cx * col[j][2];
        m2[j] = c.fy * col[j][1] + c.cy * col[j][2];
        m3[j] = col[j][2];
    }
    const double pz = p[2];
    bool culled = cull_opac || (pz <= c.znear) || ((pz * pz) <= rs2 * (au[2] * au[2] + av[2] * av[2]));
    int ilo = 0, ihi = -1, jlo = 0, jhi = -1;
    double ccx = 0.0, ccy = 0.0;
    if (!culled) {
        const double d13 = conic_dot(rs2, m1, m3), d11 = conic_dot(rs2, m1, m1);
        const double d23 = conic_dot(rs2, m2, m3), d22 = conic_dot(rs2, m2, m2);
        const double d33 = conic_dot(rs2, m3, m3);
        const double dx_ = d13 * d13 - d11 * d33, dy_ = d23 * d23 - d22 * d33;
        const double sdx = sqrt(dx_ > 0.0 ? dx_ : 0.0);
        const double sdy = sqrt(dy_ > 0.0 ? dy_ : 0.0);
        const double xa = (d13 - sdx) / d33, xb = (d13 + sdx) / d33;
        const double ya = (d23 - sdy) / d33, yb = (d23 + sdy) / d33;
        ccx = m1[2] / m3[2];
        ccy = m2[2] / m3[2];
        const double xmin = fmin(fmin(xa, xb), ccx - rf), xmax = fmax(fmax(xa, xb), ccx + rf);
        const double ymin = fmin(fmin(ya, yb), ccy - rf), ymax = fmax(fmax(ya, yb), ccy + rf);
        // numpy-style NaN propagation: any NaN operand empties the rectangle
        const bool nan = isnan(dx_) || isnan(dy_) || isnan(xa) || isnan(xb) || isnan(ya) ||
                         isnan(yb) || isnan(ccx) || isnan(ccy) || isnan(rf);
        const double flo = fmax(ceil(xmin - 0.5), 0.0), fhi = fmin(floor(xmax - 0.5), c.W - 1.0);
        const double glo = fmax(ceil(ymin - 0.5), 0.0), ghi = fmin(floor(ymax - 0.5), c.H - 1.0);
        if (nan || !(flo <= fhi) || !(glo <= ghi)) {
            culled = true;
        } else {
            ilo = (int)flo; ihi = (int)fhi; jlo = (int)glo; jhi = (int)ghi;
        }
    }
    if (culled) {
        out.tiles = 0u;
        out.key = 0xFFFFFFFFu;
        out.rx = out.ry = 0u;
        return false;
    }
    const int txlo = ilo >> tile_wl, txhi = ihi >> tile_wl, tylo = jlo >> tile_hl, tyhi = jhi >> tile_hl;
    out.tiles = (uint32_t)((txhi - txlo + 1) * (tyhi - tylo + 1));
    out.key = __float_as_uint((float)pz);
    out.rx = (uint32_t)ilo | ((uint32_t)ihi << 16);
    out.ry = (uint32_t)jlo | ((uint32_t)jhi << 16);
    // inverse homography columns: A = m2 x m3, B = m3 x m1, C = m1 x m2;
    // shifted to the float32 centre: C' = C + A cx + B cy
    double A[3], B[3], C[3];
    cross3d(m2, m3, A);
    cross3d(m3, m1, B);
    cross3d(m1, m2, C);
    const float cx32 = (float)ccx, cy32 = (float)ccy;
    double Cs[3];
    for (int i = 0; i < 3; ++i) Cs[i] = (C[i] + A[i] * (double)cx32) + B[i] * (double)cy32;
    out.geom[0] = make_float4((float)A[0], (float)A[1], (float)A[2], (float)B[0]);
    out.geom[1] = make_float4((float)B[1], (float)B[2], (float)Cs[0], (float)Cs[1]);
    out.geom[2] = make_float4((float)Cs[2], cx32, cy32, o32);
    out.geom[3] = make_float4((float)m3[0], (float)m3[1], (float)m3[2], (float)L);
    if (DEG >= 0) {
        float rgb[3];
        view_colour<DEG, SH_STEP>(mu32, cams[v].campos, shg, rgb);
        out.app[0] = make_float4(rgb[0], rgb[1], rgb[2], (float)nc[0]);
        // the pixel rectangle packed in the last two slots (column and row
        // ranges): the compositing skips, per wave, entries whose rectangle
        // misses the wave's pixels
        out.app[1] = make_float4((float)nc[1], (float)nc[2], __uint_as_float(out.rx),
                                 __uint_as_float(out.ry));
    }
    return true;
}

template <int DEG>
__device__ __forceinline__ bool project_record(int g, int v, const float* __restrict__ means,
                                               const float* __restrict__ scales, const float* __restrict__ quats,
                                               const float* __restrict__ opac, const float* __restrict__ sh,
                                               int sh_stride, float alpha_min, int tile_wl, int tile_hl,
                                               const sr_camera* __restrict__ cams, PreRec& out) {
    SurfelTerms s;
    surfel_terms(g, means, scales, quats, opac, alpha_min, s);
    return project_view<DEG, 1>(s, means + 3 * g, DEG >= 0 ? sh + (size_t)g * sh_stride * 3 : nullptr, v, tile_wl,
                                tile_hl, cams, out);
}

// Records of one workgroup staged in LDS (STAGED path).
struct PreStage {
    float4 geom[4][256];
    float4 app[2][256];
    uint2 rect[256];
    uint32_t tiles[256], key[256];
};

// One thread per (surfel g, view v), t = g * V + v: the views of one surfel
// sit in adjacent lanes, so the parameter loads of a wave are shared and the
// surfel is read from HBM once per batch; in_frustum must hold zeros on entry
// (each thread that keeps the surfel stores 1).  STAGED (V divides the
// workgroup size, so a workgroup holds 256 / V whole surfels): the records are
// assembled in LDS and written view by view, each view's records of the
// workgroup a contiguous run, instead of one scattered piece per lane.
template <int DEG, bool STAGED>
__global__ void __launch_bounds__(256)
k_preprocess(int N, const float* __restrict__ means, const float* __restrict__ scales,
             const float* __restrict__ quats, const float* __restrict__ opac,
             const float* __restrict__ sh, int sh_stride, float alpha_min,
             int tile_wl, int tile_hl, int V, const sr_camera* __restrict__ cams,
             float4* __restrict__ geom, float4* __restrict__ app, uint2* __restrict__ rect,
             uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ depth_key,
             uint8_t* __restrict__ in_frustum) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < (uint64_t)N * (uint64_t)V;
    const int g = (int)(t / (uint64_t)V);
    const int v = (int)(t - (uint64_t)g * (uint64_t)V);
    PreRec rec;
    rec.tiles = 0u;
    rec.key = 0xFFFFFFFFu;
    rec.rx = rec.ry = 0u;
    bool vis = false;
    if (live) {
        vis = project_record<DEG>(g, v, means, scales, quats, opac, sh, sh_stride, alpha_min, tile_wl, tile_hl,
                                  cams, rec);
        if (vis && in_frustum) in_frustum[g] = 1;
    }
    if (!STAGED) {
        if (!live) return;
        const size_t r = (size_t)v * N + g;
        tiles_touched[r] = rec.tiles;
        depth_key[r] = rec.key;
        rect[r] = make_uint2(rec.rx, rec.ry);
        if (!vis) return;
#pragma unroll
        for (int q = 0; q < 4; ++q) geom[4 * r + q] = rec.geom[q];
        if (DEG >= 0) {
            app[2 * r + 0] = rec.app[0];
            app[2 * r + 1] = rec.app[1];
        }
        return;
    }
    __shared__ PreStage sm;
    const int tid = threadIdx.x;
    sm.tiles[tid] = rec.tiles;
    sm.key[tid] = rec.key;
    sm.rect[tid] = make_uint2(rec.rx, rec.ry);
    if (vis) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sm.geom[q][tid] = rec.geom[q];
        if (DEG >= 0) {
            sm.app[0][tid] = rec.app[0];
            sm.app[1][tid] = rec.app[1];
        }
    }
    __syncthreads();
    // slot s = (surfel - G0) * V + view; output position p = view * ng + (surfel - G0)
    const int lv = __builtin_ctz((unsigned)V);
    const int lng = 8 - lv;                     // ng = 256 / V surfels per workgroup
    const int G0 = (int)blockIdx.x << lng;
    {
        const int vv = tid >> lng, gl = tid & ((1 << lng) - 1), s = (gl << lv) + vv, gg = G0 + gl;
        if (gg < N) {
            const size_t r = (size_t)vv * N + gg;
            tiles_touched[r] = sm.tiles[s];
            depth_key[r] = sm.key[s];
            rect[r] = sm.rect[s];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = i * 256 + tid, pp = j >> 2, q = j & 3;
        const int vv = pp >> lng, gl = pp & ((1 << lng) - 1), s = (gl << lv) + vv, gg = G0 + gl;
        if (gg < N && sm.tiles[s] != 0u) geom[4 * ((size_t)vv * N + gg) + q] = sm.geom[q][s];
    }
    if (DEG >= 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int j = i * 256 + tid, pp = j >> 1, q = j & 1;
            const int vv = pp >> lng, gl = pp & ((1 << lng) - 1), s = (gl << lv) + vv, gg = G0 + gl;
            if (gg < N && sm.tiles[s] != 0u) app[2 * ((size_t)vv * N + gg) + q] = sm.app[q][s];
        }
    }
}

// One thread per surfel, looping over the views (for batches with enough
// surfels to fill the device): the view-independent terms (unit quaternion,
// frame, cutoff radii) and the colour coefficients are evaluated and loaded
// once per surfel instead of once per (surfel, view), and the camera of an
// iteration is uniform across the wave.  Each view's records are written at
// r = v N + g, so a wave's stores of one view cover a contiguous run.  The
// records are bit for bit those of k_preprocess (the same functions).
template <int DEG>
__global__ void __launch_bounds__(256)
k_preprocess_views(int N, const float* __restrict__ means, const float* __restrict__ scales,
                   const float* __restrict__ quats, const float* __restrict__ opac,
                   const float* __restrict__ sh, int sh_stride, float alpha_min,
                   int tile_wl, int tile_hl, int V, const sr_camera* __restrict__ cams,
                   float4* __restrict__ geom, float4* __restrict__ app, uint2* __restrict__ rect,
                   uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ depth_key,
                   uint8_t* __restrict__ in_frustum) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    SurfelTerms s;
    surfel_terms(g, means, scales, quats, opac, alpha_min, s);
    const float mu32[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
    // colour coefficients: registers up to degree 1, a private LDS column per
    // thread above (48 floats at degree 3 would cut the occupancy)
    constexpr int K3 = DEG >= 0 ? 3 * (DEG + 1) * (DEG + 1) : 1;
    constexpr bool SH_LDS = DEG >= 2;
    __shared__ float s_sh[SH_LDS ? K3 : 1][SH_LDS ? 256 : 1];
    float shr[SH_LDS ? 1 : K3];
    if (DEG >= 0) {
        const float* shg = sh + (size_t)g * sh_stride * 3;
#pragma unroll
        for (int i = 0; i < K3; ++i) {
            if (SH_LDS) s_sh[i][threadIdx.x] = shg[i];
            else shr[i] = shg[i];
        }
    }
    bool any = false;
    for (int v = 0; v < V; ++v) {
        PreRec rec;
        const bool vis = SH_LDS ? project_view<DEG, 256>(s, mu32, &s_sh[0][threadIdx.x], v, tile_wl, tile_hl, cams, rec)
                                : project_view<DEG, 1>(s, mu32, shr, v, tile_wl, tile_hl, cams, rec);
        const size_t r = (size_t)v * N + g;
        tiles_touched[r] = rec.tiles;
        depth_key[r] = rec.key;
        rect[r] = make_uint2(rec.rx, rec.ry);
        if (vis) {
            any = true;
#pragma unroll
            for (int q = 0; q < 4; ++q) geom[4 * r + q] = rec.geom[q];
            if (DEG >= 0) {
                app[2 * r + 0] = rec.app[0];
                app[2 * r + 1] = rec.app[1];
            }
        }
    }
    if (any && in_frustum) in_frustum[g] = 1;
}

__global__ void k_zero_u8(uint8_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Backward of the projection: chains the per-record gradients accumulated by
// the raster backward (layout below) to the surfel parameters, summed over
// the views, and clears every accumulator it consumed.  One thread per
// surfel; the parameter gradients are added to.  With `marked`, only the
// records whose bit 31 of tiles_touched the raster backward set are read
// (and the bit is cleared): a visible record that no pixel blended holds
// zeros, and most of a batch's visible records are such (occluded).
//   grad_rec[r*24 + ...]: [0..2] dA (= sum dL/dw * dx), [3..5] dB, [6..8] dC',
//   [9..10] d centre (low-pass), [11] d opacity, [12..14] d m3,
//   [15..17] d rgb, [18..20] d normal.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cross3f(const float* a, const float* b, float* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <int DEG>
__global__ void __launch_bounds__(256)
k_preprocess_bwd(int N, const float* __restrict__ means, const float* __restrict__ scales,
                 const float* __restrict__ quats, const float* __restrict__ sh,
                 int sh_stride, int V, const sr_camera* __restrict__ cams,
                 const float4* __restrict__ geom, const float4* __restrict__ app,
                 uint32_t* __restrict__ tiles_touched, bool marked, float* __restrict__ grad_rec,
                 float* __restrict__ g_means, float* __restrict__ g_scales, float* __restrict__ g_quats,
                 float* __restrict__ g_opac, float* __restrict__ g_sh, float* __restrict__ dens_grad,
                 uint32_t* __restrict__ dens_count) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    // density-control statistic: |dL/d delta| of a screen-space translation
    // delta of the record, summed over views, and the views not culled
    float dens_sum = 0.0f;
    uint32_t dens_n = 0u;
    const float mu[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
    const float su = scales[2 * g], sv = scales[2 * g + 1];
    const float q0[4] = {quats[4 * g], quats[4 * g + 1], quats[4 * g + 2], quats[4 * g + 3]};
    const float qn = sqrtf(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    const float w = q0[0] / qn, x = q0[1] / qn, y = q0[2] / qn, z = q0[3] / qn;
    const float tu[3] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y + w * z), 2.0f * (x * z - w * y)};
    const float tv[3] = {2.0f * (x * y - w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z + w * x)};
    const float nn[3] = {2.0f * (x * z + w * y), 2.0f * (y * z - w * x), 1.0f - 2.0f * (x * x + y * y)};
    constexpr int K = (DEG + 1) * (DEG + 1);

    float dmu[3] = {0, 0, 0}, dsu = 0, dsv = 0, dopac = 0;
    float dtu[3] = {0, 0, 0}, dtv[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
    // SH gradient accumulators: registers up to degree 1, a private LDS
    // column per thread above (48 floats at degree 3 would halve occupancy)
    constexpr bool SH_LDS = DEG >= 2;
    __shared__ float s_dsh[SH_LDS ? 3 * K : 1][SH_LDS ? 256 : 1];
    float dsh[SH_LDS ? 1 : 3 * K];
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) {
        if (SH_LDS) s_dsh[i][tid] = 0.0f;
        else dsh[i] = 0.0f;
    }
    const float* shg = sh + (size_t)g * sh_stride * 3;

    // views in chunks of 32: the records' visibility and marks are read for
    // the whole chunk first (independent loads in flight), then only the
    // views that hold gradients are worked through
    for (int v0 = 0; v0 < V; v0 += 32) {
      const int vn = V - v0 < 32 ? V - v0 : 32;
      uint32_t todo = 0u;
      if (tiles_touched) {
#pragma unroll 8
        for (int j = 0; j < 32; ++j) {
            if (j >= vn) break;
            const size_t r = (size_t)(v0 + j) * N + g;
            const uint32_t tt = tiles_touched[r];
            if ((tt & 0x7FFFFFFFu) == 0u) continue;          // culled in this view
            dens_n += 1u;
            if (marked) {
                // only records the compositing backward marked hold gradients
                if ((tt >> 31) == 0u) continue;
                tiles_touched[r] = tt & 0x7FFFFFFFu;
            }
            todo |= 1u << j;
        }
      } else {
        dens_n += (uint32_t)vn;
        todo = vn == 32 ? 0xFFFFFFFFu : ((1u << vn) - 1u);
      }
      while (todo != 0u) {
        const int v = v0 + __builtin_ctz(todo);
        todo &= todo - 1u;
        const size_t r = (size_t)v * N + g;
        float* gr = grad_rec + r * SR_GRAD_STRIDE;
        float G[kNumGrad];
        bool any = false;
        for (int i = 0; i < kNumGrad; ++i) { G[i] = gr[i]; any |= (G[i] != 0.0f); }
        if (!any) continue;
        if (dens_grad) {
            // w = A dx + B dy + C' with dx = x - c: translating by delta shifts
            // dx by -delta, so dL/d delta = (low-pass terms) - (A, B) . dL/dC'
            const float4 h0 = geom[4 * r], h1 = geom[4 * r + 1];
            const float sx = G[9] - (h0.x * G[6] + h0.y * G[7] + h0.z * G[8]);
            const float sy = G[10] - (h0.w * G[6] + h1.x * G[7] + h1.y * G[8]);
            dens_sum += sqrtf(sx * sx + sy * sy);
        }
        // consume: leave the accumulator zero for the next backward
        for (int i = 0; i < kNumGrad; ++i) gr[i] = 0.0f;
        const sr_camera& cam = cams[v];
        float R[9], t[3];
        for (int i = 0; i < 3; ++i) {
            R[3 * i] = cam.viewmat[4 * i]; R[3 * i + 1] = cam.viewmat[4 * i + 1];
            R[3 * i + 2] = cam.viewmat[4 * i + 2]; t[i] = cam.viewmat[4 * i + 3];
        }
        float p[3], Rtu[3], Rtv[3], Rn[3], au[3], av[3];
        for (int i = 0; i < 3; ++i) {
            p[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + t[i];
            Rtu[i] = R[3 * i] * tu[0] + R[3 * i + 1] * tu[1] + R[3 * i + 2] * tu[2];
            Rtv[i] = R[3 * i] * tv[0] + R[3 * i + 1] * tv[1] + R[3 * i + 2] * tv[2];
            Rn[i] = R[3 * i] * nn[0] + R[3 * i + 1] * nn[1] + R[3 * i + 2] * nn[2];
            au[i] = su * Rtu[i];
            av[i] = sv * Rtv[i];
        }
        const float* col[3] = {au, av, p};
        float m1[3], m2[3], m3[3];
        for (int j = 0; j < 3; ++j) {
            m1[j] = cam.fx * col[j][0] + cam.cx * col[j][2];
            m2[j] = cam.fy * col[j][1] + cam.cy * col[j][2];
            m3[j] = col[j][2];
        }
        const float4 g2 = geom[4 * r + 2];
        const float ccx = g2.y, ccy = g2.z;
        // undo the centre shift: w = A x + B y + C in absolute pixels
        float dA[3], dB[3], dC[3];
        for (int i = 0; i < 3; ++i) {
            dC[i] = G[6 + i];
            dA[i] = G[0 + i] + ccx * dC[i];
            dB[i] = G[3 + i] + ccy * dC[i];
        }
        float dm1[3], dm2[3], dm3[3] = {G[12], G[13], G[14]}, tmp[3];
        // A = m2 x m3, B = m3 x m1, C = m1 x m2
        cross3f(dB, m3, dm1); cross3f(m2, dC, tmp);
        for (int i = 0; i < 3; ++i) dm1[i] += tmp[i];
        cross3f(m3, dA, dm2); cross3f(dC, m1, tmp);
        for (int i = 0; i < 3; ++i) dm2[i] += tmp[i];
        cross3f(dA, m2, tmp);
        for (int i = 0; i < 3; ++i) dm3[i] += tmp[i];
        cross3f(m1, dB, tmp);
        for (int i = 0; i < 3; ++i) dm3[i] += tmp[i];
        // centre c = (m1_2 / m3_2, m2_2 / m3_2), low-pass branch
        {
            const float iz = 1.0f / m3[2];
            dm1[2] += G[9] * iz;
            dm2[2] += G[10] * iz;
            dm3[2] -= (G[9] * m1[2] + G[10] * m2[2]) * iz * iz;
        }
        // columns (a_u, a_v, p) of M = K [a_u a_v p]
        float dcol[3][3];
        for (int j = 0; j < 3; ++j) {
            dcol[j][0] = cam.fx * dm1[j];
            dcol[j][1] = cam.fy * dm2[j];
            dcol[j][2] = cam.cx * dm1[j] + cam.cy * dm2[j] + dm3[j];
        }
        // p = R mu + t ; a_u = s_u R t_u ; a_v = s_v R t_v
        for (int k = 0; k < 3; ++k) {
            float rp = 0, ru = 0, rv = 0;
            for (int i = 0; i < 3; ++i) {
                rp += R[3 * i + k] * dcol[2][i];
                ru += R[3 * i + k] * dcol[0][i];
                rv += R[3 * i + k] * dcol[1][i];
            }
            dmu[k] += rp;
            dtu[k] += su * ru;
            dtv[k] += sv * rv;
        }
        dsu += Rtu[0] * dcol[0][0] + Rtu[1] * dcol[0][1] + Rtu[2] * dcol[0][2];
        dsv += Rtv[0] * dcol[1][0] + Rtv[1] * dcol[1][1] + Rtv[2] * dcol[1][2];
        // normal n_c = sign R n (sign chosen by the projection)
        const float4 a0 = app[2 * r + 0], a1 = app[2 * r + 1];
        const float ncs[3] = {a0.w, a1.x, a1.y};
        const float sgn = (ncs[0] * Rn[0] + ncs[1] * Rn[1] + ncs[2] * Rn[2]) < 0.0f ? -1.0f : 1.0f;
        for (int k = 0; k < 3; ++k)
            dn[k] += sgn * (R[k] * G[18] + R[3 + k] * G[19] + R[6 + k] * G[20]);
        dopac += G[11];
        // colour: rgb = max(0, sum Y f + 1/2), clamped channels pass no gradient
        const float rgb[3] = {a0.x, a0.y, a0.z};
        const float dr[3] = {rgb[0] > 0.0f ? G[15] : 0.0f, rgb[1] > 0.0f ? G[16] : 0.0f,
                             rgb[2] > 0.0f ? G[17] : 0.0f};
        if (dr[0] != 0.0f || dr[1] != 0.0f || dr[2] != 0.0f) {
            const float* cp = cam.campos;
            float d[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
            const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const float il = 1.0f / len;
            d[0] *= il; d[1] *= il; d[2] *= il;
            float Y[16], gx[16], gy[16], gz[16];
            sh_basis(DEG, d[0], d[1], d[2], Y);
            sh_basis_grad(DEG, d[0], d[1], d[2], gx, gy, gz);
            float dd[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float f0 = shg[3 * k], f1 = shg[3 * k + 1], f2 = shg[3 * k + 2];
                if (SH_LDS) {
                    s_dsh[3 * k + 0][tid] += Y[k] * dr[0];
                    s_dsh[3 * k + 1][tid] += Y[k] * dr[1];
                    s_dsh[3 * k + 2][tid] += Y[k] * dr[2];
                } else {
                    dsh[3 * k + 0] += Y[k] * dr[0];
                    dsh[3 * k + 1] += Y[k] * dr[1];
                    dsh[3 * k + 2] += Y[k] * dr[2];
                }
                const float s = f0 * dr[0] + f1 * dr[1] + f2 * dr[2];
                dd[0] += s * gx[k];
                dd[1] += s * gy[k];
                dd[2] += s * gz[k];
            }
            const float dp = d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2];
            for (int k = 0; k < 3; ++k) dmu[k] += (dd[k] - d[k] * dp) * il;
        }
      }
    }
    // rotation matrix R(q^) with columns (t_u, t_v, n): dR_ik
    const float d00 = dtu[0], d10 = dtu[1], d20 = dtu[2];
    const float d01 = dtv[0], d11 = dtv[1], d21 = dtv[2];
    const float d02 = dn[0], d12 = dn[1], d22 = dn[2];
    float dq[4];
    dq[0] = 2.0f * (-z * d01 + y * d02 + z * d10 - x * d12 - y * d20 + x * d21);
    dq[1] = 2.0f * (y * d01 + z * d02 + y * d10 - 2.0f * x * d11 - w * d12 + z * d20 + w * d21 - 2.0f * x * d22);
    dq[2] = 2.0f * (-2.0f * y * d00 + x * d01 + w * d02 + x * d10 + z * d12 - w * d20 + z * d21 - 2.0f * y * d22);
    dq[3] = 2.0f * (-2.0f * z * d00 - w * d01 + x * d02 + w * d10 - 2.0f * z * d11 + y * d12 + x * d20 + y * d21);
    const float qh[4] = {w, x, y, z};
    const float dot = qh[0] * dq[0] + qh[1] * dq[1] + qh[2] * dq[2] + qh[3] * dq[3];
    for (int i = 0; i < 4; ++i) g_quats[4 * g + i] += (dq[i] - qh[i] * dot) / qn;
    for (int i = 0; i < 3; ++i) g_means[3 * g + i] += dmu[i];
    g_scales[2 * g] += dsu;
    g_scales[2 * g + 1] += dsv;
    g_opac[g] += dopac;
    float* gs = g_sh + (size_t)g * sh_stride * 3;
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) gs[i] += SH_LDS ? s_dsh[i][tid] : dsh[SH_LDS ? 0 : i];
    if (dens_grad) dens_grad[g] += dens_sum;
    if (dens_count) dens_count[g] += dens_n;
}

}  // namespace

hipError_t launch_preprocess(const sr_config& cfg, int N, const float* means, const float* scales,
                             const float* quats, const float* opac, const float* sh, int V,
                             const sr_camera* cams_dev, float* geom, float* app, uint16_t* rect,
                             uint32_t* tiles_touched, uint32_t* depth_key, uint8_t* in_frustum,
                             hipStream_t stream) {
    if (N == 0) return hipSuccess;
    // the supported tile shapes are powers of two
    if ((cfg.tile_w & (cfg.tile_w - 1)) != 0 || (cfg.tile_h & (cfg.tile_h - 1)) != 0) return hipErrorInvalidValue;
    if (in_frustum && !(cfg.flags & SR_FLAG_ACCUMULATE))
        hipLaunchKernelGGL(k_zero_u8, dim3((N + 255) / 256), dim3(256), 0, stream, in_frustum, N);
    const uint64_t threads = (uint64_t)N * (uint64_t)V;
    if (threads == 0) return hipGetLastError();
    dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    const int deg = app ? cfg.sh_degree : -1;
    // enough surfels for several workgroups of 256 per compute unit: one
    // thread per surfel looping over the views; else one thread per (surfel,
    // view), with staged writes when V divides the workgroup size (V a power
    // of two <= 256)
    const bool per_surfel = N >= kPreprocessLoopMinSurfels || V == 1;
    const int twl = __builtin_ctz((unsigned)cfg.tile_w), thl = __builtin_ctz((unsigned)cfg.tile_h);
    const bool staged = V <= 256 && (256 % V) == 0;
#define SR_PRE(D)                                                                                                 \
    if (per_surfel)                                                                                               \
        hipLaunchKernelGGL((k_preprocess_views<D>), dim3((N + 255) / 256), block, 0, stream, N, means, scales,    \
                           quats, opac, sh, cfg.sh_stride, cfg.alpha_min, twl, thl, V, cams_dev,                  \
                           (float4*)geom, (float4*)app, (uint2*)rect, tiles_touched, depth_key, in_frustum);      \
    else if (staged)                                                                                              \
        hipLaunchKernelGGL((k_preprocess<D, true>), grid, block, 0, stream, N, means, scales, quats, opac, sh,    \
                           cfg.sh_stride, cfg.alpha_min, twl, thl, V, cams_dev, (float4*)geom,                    \
                           (float4*)app, (uint2*)rect, tiles_touched, depth_key, in_frustum);                     \
    else                                                                                                          \
        hipLaunchKernelGGL((k_preprocess<D, false>), grid, block, 0, stream, N, means, scales, quats, opac, sh,   \
                           cfg.sh_stride, cfg.alpha_min, twl, thl, V, cams_dev, (float4*)geom,                    \
                           (float4*)app, (uint2*)rect, tiles_touched, depth_key, in_frustum)
    switch (deg) {
        case 0: SR_PRE(0); break;
        case 1: SR_PRE(1); break;
        case 2: SR_PRE(2); break;
        case 3: SR_PRE(3); break;
        default: SR_PRE(-1); break;
    }
#undef SR_PRE
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const sr_config& cfg, int N, const float* means, const float* scales,
                                 const float* quats, const float* sh, int V, const sr_camera* cams_dev,
                                 const float* geom, const float* app, uint32_t* tiles_touched,
                                 float* grad_rec, float* g_means, float* g_scales, float* g_quats,
                                 float* g_opac, float* g_sh, float* dens_grad, uint32_t* dens_count,
                                 hipStream_t stream) {
    if (N == 0) return hipSuccess;
    dim3 grid((N + 255) / 256), block(256);
    const bool marked = tiles_touched && (cfg.flags & SR_FLAG_MARKED_GRADIENTS);
#define SR_PREB(D)                                                                                          \
    hipLaunchKernelGGL(k_preprocess_bwd<D>, grid, block, 0, stream, N, means, scales, quats, sh,            \
                       cfg.sh_stride, V, cams_dev, (const float4*)geom, (const float4*)app, tiles_touched,   \
                       marked, grad_rec, g_means, g_scales, g_quats, g_opac, g_sh, dens_grad, dens_count)
    switch (cfg.sh_degree) {
        case 0: SR_PREB(0); break;
        case 1: SR_PREB(1); break;
        case 2: SR_PREB(2); break;
        default: SR_PREB(3); break;
    }
#undef SR_PREB
    return hipGetLastError();
}

}  // namespace sr
