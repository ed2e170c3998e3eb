// Front-to-back alpha compositing of surfels per tile, its recompute-based
// backward, and the occlusion statistics of the pruning pass.
//
// Section 4.3: a pixel blends its assigned Gaussians front to back,
// accumulating colour and opacity, and stops once the accumulated opacity
// reaches a threshold close to one or the list is exhausted; a Gaussian that
// takes part in the blending of a pixel is "used" (visible).  Section 4.2
// (Eq. 1) consumes the accumulated alpha; Eq. 3's 2DGS regularisers consume
// depth, normal and distortion.
//
// One workgroup per (view, tile) over all views of the batch in a single
// launch; one thread per pixel; surfel records are staged in LDS one batch
// per workgroup-size entries; every pair is evaluated with the shared
// eval_test()/eval_finish() so that forward, backward and pruning take identical
// decisions.
#include <mutex>

#include <type_traits>

#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr int kWaveBlock = 8;   // side of the square block of pixels one wave covers

// Square root and reciprocal for the culling bounds: the hardware estimates
// refined by one Newton step, far more accurate than the culling's 1e-3
// margins need and a fraction of the instructions of the correctly rounded
// operations.  x >= 0 for the root: below 1e-300 it is taken as 0 (an error
// under 1e-150 px), an infinite x stays infinite; the reciprocal is taken of
// positive normal numbers.
__device__ __forceinline__ double cull_sqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);                 // 1/sqrt(x), refined as y (3 - x y^2) / 2
    const double r = x * (y * (1.5 - 0.5 * x * y * y));
    return x > 1e-300 ? (x <= 1.7e308 ? r : x) : 0.0;
}
__device__ __forceinline__ double cull_rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return r * (2.0 - x * r);
}

// Global tile id of this workgroup; pixel coordinates of this thread; the
// run [start, start + n) of the tile's binning group.
struct TileCtx {
    int tile, v, W, H, ix, iy;
    int tx0, ty0;    // first pixel column and row of the tile
    int sx, sy;      // tile coordinates inside its binning group
    bool inside;
    int64_t pix_off;
    uint32_t start, n;
    float bg[3];
};

template <int TW, int TH>
// order (optional): the tile of each workgroup, a permutation of the tile ids
// (heaviest first); an id beyond the grid marks the workgroup idle
// (t.n = 0, nothing inside).
__device__ __forceinline__ void tile_ctx(const sr_camera* __restrict__ cams, int V,
                                         const uint2* __restrict__ ranges, TileCtx& t,
                                         const uint32_t* __restrict__ order = nullptr) {
    int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    bool idle = false;
    if (order) {
        const uint32_t o = order[blockIdx.x];
        idle = o >= gridDim.x;
        tile = idle ? 0 : (int)o;
    }
    t.tile = tile;
    t.v = view_of_tile(cams, V, tile);
    const sr_camera& c = cams[t.v];
    const int local = tile - c.tile_offset;
    const int ty = local / c.tiles_x, tx = local - ty * c.tiles_x;
    t.W = c.width;
    t.H = c.height;
    // wave w covers the 8x8 block (w % (TW / 8), w / (TW / 8)) of the tile
    constexpr int WB = kWaveBlock;
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    t.ix = tx * TW + (w % (TW / WB)) * WB + (l % WB);
    t.iy = ty * TH + (w / (TW / WB)) * WB + l / WB;
    t.tx0 = tx * TW;
    t.ty0 = ty * TH;
    t.sx = tx % SR_TILE_GROUP;
    t.sy = ty % SR_TILE_GROUP;
    t.inside = !idle && t.ix < t.W && t.iy < t.H;
    t.pix_off = c.pix_offset;
    t.bg[0] = c.bg[0]; t.bg[1] = c.bg[1]; t.bg[2] = c.bg[2];
    const uint2 rg = ranges[tile];
    t.start = rg.x;
    t.n = idle ? 0u : rg.y - rg.x;
}

constexpr int kMaxWaves = 8;    // waves per workgroup (tiles of up to 512 pixels)

// Five waves per SIMD: the register budget (at most 96 VGPRs, no spills)
// that keeps the compositing kernels issue-bound; the compiler would
// otherwise spend up to 104 registers and drop to four.
#define SR_RASTER_OCCUPANCY __attribute__((amdgpu_waves_per_eu(5)))

// MODE bits: 1 shade (colour, depth, normal, distortion outputs), 2 occlusion
// statistics, 4 count reached/blended pairs (work accounting), 8 median depth
// (the 2DGS surface depth: the depth of the last blended entry that starts
// with transmittance above 1/2) with the 1-based list index of that entry,
// 16 pixel rectangles read from the rectangle array (statistics without
// shading: no appearance records to take them from).
constexpr int kShade = 1, kStats = 2, kCount = 4, kMedian = 8, kRect = 16, kHits = 32;

// Per-wave culling.  Every wave of a tile covers an 8x8 block of its pixels
// (wave w: block column w % (TW / 8), block row w / (TW / 8)); a square
// footprint has the shortest boundary for its 64 pixels, so fewer of a
// wave's lanes sit outside the splats it works through than with a strip of
// rows.  When an entry is staged, its thread works out which blocks it can
// reach, one bit per wave; each wave then tests 64 staged entries at once
// with one ballot of its bit and walks only the set bits of that mask, so
// skipped entries cost no per-entry instructions.  A block is reached when
// the entry's pixel rectangle (packed in the last two slots of the appearance
// record) meets it and the y-range, within the block's columns that the
// rectangle meets, of the entry's cutoff conic or of its low-pass disc meets
// the block's rows:
//   surface  Q = (1 - tau)(w0^2 + w1^2) - 2 L (1 + tau) w2^2 <= 0 with
//            w = A dx + B dy + C' (the pass test of eval_test with a relative
//            slack tau): for an ellipse, Q(x, .) <= 0 is the interval between
//            the roots of a quadratic in y, whose lower end is convex and
//            upper end concave in x, so their extremes over the columns are
//            at the ellipse's lowest and highest points clamped to the
//            columns; any other conic reaches every block;
//   disc     dx^2 + dy^2 <= L (1 + tau).
// Float64, with a 1e-3 pixel margin on the columns and rows: an entry is
// skipped only where the exact test fails by a relative margin, and forward
// and backward skip the same entries.
template <int TW, int NW>
__device__ __forceinline__ uint32_t wave_bits(const float4& g0, const float4& g1, const float4& g2, float Lf,
                                              const float4& a1, int tx0, int ty0) {
    constexpr int WB = kWaveBlock;
    static_assert(TW % WB == 0 && NW % (TW / WB) == 0, "waves cover whole 8x8 blocks of the tile");
    constexpr int BX = TW / WB, BY = NW / BX;     // blocks per tile row and column
    constexpr double tau = 1e-3, mg = 1e-3;
    const uint32_t rx = __float_as_uint(a1.z), ry = __float_as_uint(a1.w);
    const int ilo = (int)(rx & 0xffffu), ihi = (int)(rx >> 16), jlo = (int)(ry & 0xffffu), jhi = (int)(ry >> 16);
    const double cx = g2.y, cy = g2.z, L = Lf;
    // the conic's coefficients, independent of the columns
    const double s01 = 1.0 - tau, s2 = -2.0 * L * (1.0 + tau);
    const double a0 = g0.x, a1x = g0.y, a2 = g0.z, b0 = g0.w, b1 = g1.x, b2 = g1.y, c0 = g1.z, c1 = g1.w,
                 c2 = g2.x;
    // Q = P x^2 + 2 R x y + S y^2 + 2 U x + 2 W y + K
    const double P = s01 * (a0 * a0 + a1x * a1x) + s2 * (a2 * a2);
    const double R = s01 * (a0 * b0 + a1x * b1) + s2 * (a2 * b2);
    const double S = s01 * (b0 * b0 + b1 * b1) + s2 * (b2 * b2);
    const double U = s01 * (a0 * c0 + a1x * c1) + s2 * (a2 * c2);
    const double W = s01 * (b0 * c0 + b1 * c1) + s2 * (b2 * c2);
    const double K = s01 * (c0 * c0 + c1 * c1) + s2 * (c2 * c2);
    const double al = P * S - R * R;
    const bool ellipse = P > 0.0 && S > 0.0 && al > 0.0;
    // discriminant in y of Q(x, .): D(x) = -al x^2 + 2 be x + ga, >= 0 on the ellipse's columns
    const double be = R * W - S * U, ga = W * W - S * K;
    const double ex = be * be + al * ga;
    // the ellipse's columns [xl, xr] (empty unless ex >= 0) and the x of its
    // lowest and highest points (on P x + R y + U = 0, y roots of the
    // discriminant in x)
    double xl = 1.0, xr = -1.0, xb0 = 0.0, xt0 = 0.0, iS = 0.0;
    if (ellipse && ex >= 0.0) {
        const double ia = cull_rcp(al), sx = cull_sqrt(ex);
        xl = (be - sx) * ia;
        xr = (be + sx) * ia;
        const double bp = R * U - P * W, gp = U * U - P * K;
        const double sy = cull_sqrt(fmax(bp * bp + al * gp, 0.0));
        const double iP = cull_rcp(P);
        iS = cull_rcp(S);
        xb0 = -(R * ((bp - sy) * ia) + U) * iP;
        xt0 = -(R * ((bp + sy) * ia) + U) * iP;
    }
    uint32_t bits = 0u;
#pragma unroll 1
    for (int bx = 0; bx < BX; ++bx) {
        const int k0 = tx0 + bx * WB, k1 = k0 + WB - 1;
        const int clo = ilo > k0 ? ilo : k0, chi = ihi < k1 ? ihi : k1;
        if (clo > chi) continue;
        const double X0 = (clo + 0.5) - cx - mg, X1 = (chi + 0.5) - cx + mg;
        // disc: |dy| <= hd
        const double xd = fmin(fmax(0.0, X0), X1);
        const double hd2 = L * (1.0 + tau) - xd * xd;
        const double hd = hd2 >= 0.0 ? cull_sqrt(hd2) : -1.0;
        // surface: y-range [ylo, yhi] over these columns (empty when ylo > yhi)
        double ylo = -1e300, yhi = 1e300;
        if (ellipse) {
            ylo = 1.0;
            yhi = -1.0;
            const double xa = fmax(X0, xl), xb = fmin(X1, xr);
            if (xa <= xb) {
                const double xbot = fmin(fmax(xb0, xa), xb);
                const double xtop = fmin(fmax(xt0, xa), xb);
                const double db = fmax((-al * xbot + 2.0 * be) * xbot + ga, 0.0);
                const double dt = fmax((-al * xtop + 2.0 * be) * xtop + ga, 0.0);
                ylo = (-(R * xbot + W) - cull_sqrt(db)) * iS;
                yhi = (-(R * xtop + W) + cull_sqrt(dt)) * iS;
            }
        }
#pragma unroll
        for (int by = 0; by < BY; ++by) {
            const int r0 = ty0 + by * WB, r1 = r0 + WB - 1;
            const int lo = jlo > r0 ? jlo : r0, hi = jhi < r1 ? jhi : r1;
            if (lo > hi) continue;
            const double Y0 = (lo + 0.5) - cy - mg, Y1 = (hi + 0.5) - cy + mg;
            const bool disc = hd >= 0.0 && Y0 <= hd && Y1 >= -hd;
            const bool surf = ylo <= Y1 && yhi >= Y0;
            if (disc || surf) bits |= 1u << (by * BX + bx);
        }
    }
    return bits;
}

// Mask of the entries of run c (of 64) whose wave bit (kept in the last slot
// of the staged appearance record) is set for this wave.
__device__ __forceinline__ uint64_t wave_live_mask(const float4* __restrict__ a1, int c, int cnt) {
    const int k = c * 64 + __lane_id();
    const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6;
    return ballot64(k < cnt && ((__float_as_uint(a1[k].w) >> w) & 1u));
}

// The same for the slots [lo, hi), keeping only run positions below maxpos.
__device__ __forceinline__ uint64_t wave_live_mask_from(const float4* __restrict__ a1, int c, int lo, int hi,
                                                        uint32_t maxpos) {
    const int k = c * 64 + __lane_id();
    const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6;
    bool live = k >= lo && k < hi;
    if (live) {
        const float4 r = a1[k];
        live = ((__float_as_uint(r.w) >> w) & 1u) && __float_as_uint(r.z) < maxpos;
    }
    return ballot64(live);
}

// Wave bits of the staged entries kept from the forward to the backward of
// the fused step (LDS, 4 bits per run position, 16 bytes per thread of the
// workgroup: positions below 32 per thread; the backward recomputes the bits
// of later positions).  The backward stages only positions the forward
// staged (below the largest last contributor), so every cached position it
// reads was written.
template <int NT>
struct BitCache {
    static constexpr int kWords = 4 * NT;
    static constexpr uint32_t kPos = 8u * kWords;
};

template <int NT>
__device__ __forceinline__ void bitcache_put(uint32_t* c, uint32_t jpos, uint32_t bits) {
    if (jpos < BitCache<NT>::kPos) atomicOr(&c[jpos >> 3], bits << ((jpos & 7u) << 2));
}

// Per-pixel state at the end of the forward pass.
struct PixFwd {
    float T, C0, C1, C2, N0, N1, N2, S0, S1, S2, zref, zmed;
    uint32_t last, kmed;
};

// LDS staging of the forward: NT records per batch.
template <int NT, int MODE>
struct FwdSmem {
    float4 g[kGeomF4][NT];
    // appearance (shading) in a[0], a[1].xy; the run position of the entry in
    // a[1].z and the wave bits in a[1].w in every mode
    float4 a[kAppF4][NT];
    uint32_t id[(MODE & (kStats | kHits)) ? NT : 1];
    // occlusion statistics of the batch's entries over the workgroup's waves
    // (hits, then with kStats the max alpha and max weight bits), added to
    // the global ones once per (tile, entry) at the end of the batch
    uint32_t st[(MODE & kStats) ? 3 : 1][(MODE & (kStats | kHits)) ? NT : 1];
    uint32_t wcnt[NT / 64 + 1];   // gathering: members per wave, then the resume position
};

// LDS staging and per-record accumulators of the backward.
template <int BATCH>
struct BwdSmem {
    float4 g[kGeomF4][BATCH];
    float4 a[kAppF4][BATCH];      // as in the forward: a[1].z run position, a[1].w wave bits
    uint32_t rec[BATCH];
    float acc[BATCH][kNumGrad];
    uint32_t maxn;
    uint32_t wcnt[kMaxWaves + 1];
};

// Gathering of a batch from the tile's group run: the NT threads examine NT
// run positions at once, keep the entries whose sub-rectangle covers the
// tile, and place them in consecutive batch slots by a block-wide rank
// (wave ballots, per-wave counts in LDS).  With ASC the slots [fill, cap)
// receive the members of [pos, pos + NT) in run order; otherwise slots
// (cap - 1 - fill) downwards receive the members of [pos - NT, pos), highest
// position first.  A round that overfills the batch stops after the last
// member placed and reports where the next batch resumes.  Returns the
// number of members placed in this round; block-uniform.
template <int NT, bool ASC>
__device__ __forceinline__ int gather_round(const TileCtx& t, const uint32_t* __restrict__ vals, int64_t pos,
                                            int fill, int cap, float4* __restrict__ a0, float4* __restrict__ a1,
                                            uint32_t* wcnt, int64_t& next) {
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int64_t j = ASC ? pos + tid : pos - NT + tid;
    const bool in = ASC ? j < (int64_t)t.n : j >= 0;
    const uint32_t gv = in ? vals[t.start + (uint32_t)j] : 0u;
    const bool mem = in && inst_covers(gv, t.sx, t.sy);
    const uint64_t bm = ballot64(mem);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) wcnt[w] = (uint32_t)__popcll(bm);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const int c = (int)wcnt[i];
        before += i < w ? c : 0;
        tot += c;
    }
    const int r_asc = before + __popcll(bm & lt);
    const int rank = ASC ? r_asc : tot - 1 - r_asc;          // order of placement
    const int taken = fill + rank;
    if (mem && taken < cap) {
        const int slot = ASC ? taken : cap - 1 - taken;
        a0[slot].x = __uint_as_float(gv);
        a1[slot].z = __uint_as_float((uint32_t)j);
        if (taken == cap - 1 && fill + tot > cap) wcnt[NT / 64] = (uint32_t)(ASC ? j + 1 : j);
    }
    __syncthreads();
    if (fill + tot <= cap) {
        next = ASC ? pos + NT : (pos - NT > 0 ? pos - NT : 0);
    } else {
        next = (int64_t)wcnt[NT / 64];
        tot = cap - fill;
    }
    __syncthreads();                                          // wcnt is reused by the next round
    return tot;
}

// Front to back over the tile list; every thread owns one pixel.
template <int TW, int NT, int MODE>
__device__ __forceinline__ void fwd_tile(const TileCtx& t, float px, float py, int N, const float4* __restrict__ geom,
                                         const float4* __restrict__ app, const uint2* __restrict__ rect,
                                         const uint32_t* __restrict__ vals, const RasterConsts& rc,
                                         FwdSmem<NT, MODE>& sm, PixFwd& st,
                                         uint32_t* __restrict__ hits, float* __restrict__ max_alpha,
                                         float* __restrict__ max_weight, uint64_t& n_reached, uint64_t& n_blended,
                                         uint64_t& n_witer, uint64_t& n_wblend, uint64_t& n_upto_last,
                                         uint32_t* bitcache = nullptr) {
    static_assert(NT / 64 <= 4, "four wave bits per cached entry");
    constexpr bool SHADE = (MODE & kShade) != 0;
    constexpr bool STATS = (MODE & kStats) != 0;              // hits and the two maxima
    constexpr bool HITS = STATS || (MODE & kHits) != 0;       // hits (blended pixels per surfel)
    constexpr bool COUNT = (MODE & kCount) != 0;
    constexpr bool MEDIAN = (MODE & kMedian) != 0;
    // the pixel rectangles are staged (with the appearance records, or from
    // the rectangle array): cull per wave
    constexpr bool RECT = (MODE & kRect) != 0 && !SHADE && !COUNT;
    constexpr bool CULL = SHADE || COUNT || RECT;
    uint32_t n_eval = 0, n_eval_last = 0;     // COUNT: entries tested by this pixel, up to its last blend
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    st.T = 1.0f;
    st.C0 = st.C1 = st.C2 = st.N0 = st.N1 = st.N2 = st.S0 = st.S1 = st.S2 = st.zref = st.zmed = 0.f;
    st.last = st.kmed = 0;
    uint32_t px_live = t.inside ? 1u : 0u;    // 0 once the pixel has terminated (or lies outside)
    constexpr bool PLAIN = !COUNT && !HITS;
    // statistics of the previous batch's entries: every thread adds its own
    // slot to the global arrays (after a barrier), before the slot is reused
    int prev_cnt = 0;
    auto flush = [&]() {
        if (tid < prev_cnt && sm.st[0][tid] != 0u) {
            const uint32_t g = sm.id[tid];
            atomicAdd(&hits[g], sm.st[0][tid]);
            if (STATS) {
                atomicMax((uint32_t*)&max_alpha[g], sm.st[1][tid]);
                atomicMax((uint32_t*)&max_weight[g], sm.st[2][tid]);
            }
        }
    };
    // batches of up to NT entries of the tile, gathered from its group's run
    int64_t pos = 0;
    while (pos < (int64_t)t.n) {
        if (__syncthreads_and(px_live == 0u)) break;
        if (HITS) flush();
        int cnt = 0;
        while (cnt < NT && pos < (int64_t)t.n) {
            int64_t next;
            cnt += gather_round<NT, true>(t, vals, pos, cnt, NT, sm.a[0], sm.a[1], sm.wcnt, next);
            pos = next;
        }
        if (tid < cnt) {
            const uint32_t gv = __float_as_uint(sm.a[0][tid].x);
            const uint32_t jpos = __float_as_uint(sm.a[1][tid].z);
            const uint32_t g = gv & kInstIdMask;
            const size_t r = (size_t)t.v * N + g;
            float4 gq[kGeomF4];
#pragma unroll
            for (int q = 0; q < kGeomF4; ++q) {
                gq[q] = geom[kGeomF4 * r + q];
                sm.g[q][tid] = gq[q];
            }
            uint32_t bits = (1u << (NT / 64)) - 1u;
            float2 n12 = make_float2(0.f, 0.f);
            if (RECT) {
                // ushort4 rectangle (x_lo, x_hi, y_lo, y_hi) read as two packed ranges
                const uint2 rr = rect[r];
                const float4 a1 = make_float4(0.f, 0.f, __uint_as_float(rr.x), __uint_as_float(rr.y));
                bits = wave_bits<TW, NT / 64>(gq[0], gq[1], gq[2], gq[3].w, a1, t.tx0, t.ty0);
            } else if (CULL) {
                const float4 a0 = app[kAppF4 * r], a1 = app[kAppF4 * r + 1];
                // the appearance is stored first: fewer registers live across the bounds
                sm.a[0][tid] = a0;
                n12 = make_float2(a1.x, a1.y);
                reinterpret_cast<float2*>(&sm.a[1][tid])[0] = n12;
                bits = wave_bits<TW, NT / 64>(gq[0], gq[1], gq[2], gq[3].w, a1, t.tx0, t.ty0);
                if (bitcache) bitcache_put<NT>(bitcache, jpos, bits);
            }
            // the run position and the wave bits replace the packed rectangle
            if (CULL && !RECT)
                reinterpret_cast<float2*>(&sm.a[1][tid])[1] = make_float2(__uint_as_float(jpos), __uint_as_float(bits));
            else
                sm.a[1][tid] = make_float4(n12.x, n12.y, __uint_as_float(jpos), __uint_as_float(bits));
            if (HITS) {
                sm.id[tid] = g;
                sm.st[0][tid] = 0u;
            }
            if (STATS) {
                sm.st[1][tid] = 0u;
                sm.st[2][tid] = 0u;
            }
        }
        __syncthreads();
        bool wave_done = ballot64(px_live != 0u) == 0ull;
        for (int c = 0; c * 64 < cnt && !wave_done; ++c) {
          uint64_t live = wave_live_mask(sm.a[1], c, cnt);
          // HITS: this wave's blended pixels of entry c * 64 + lane
          uint32_t my_hits = 0;
          while (live != 0ull) {
            const int bit = (int)__builtin_ctzll(live);
            const int k = c * 64 + bit;
            live &= live - 1ull;
            PairEval e;
            const float4 g2 = sm.g[2][k], g3 = sm.g[3][k];
            eval_test(sm.g[0][k], sm.g[1][k], g2, g3, px, py, e);
            // blends entry k into the pixel state (before the transmittance update)
            auto accumulate = [&](float wgt) {
                // the depth reference of the distortion sums is the depth of
                // the pixel's first blended entry: T is exactly 1 until then
                // (every blended alpha is at least alpha_min)
                st.zref = st.T == 1.0f ? e.z : st.zref;
                const float zs = e.z - st.zref;
                if (SHADE) {
                    const float4 a0 = sm.a[0][k], a1 = sm.a[1][k];
                    st.C0 = __builtin_fmaf(wgt, a0.x, st.C0);
                    st.C1 = __builtin_fmaf(wgt, a0.y, st.C1);
                    st.C2 = __builtin_fmaf(wgt, a0.z, st.C2);
                    st.N0 = __builtin_fmaf(wgt, a0.w, st.N0);
                    st.N1 = __builtin_fmaf(wgt, a1.x, st.N1);
                    st.N2 = __builtin_fmaf(wgt, a1.y, st.N2);
                }
                st.S0 += wgt;
                st.S1 = __builtin_fmaf(wgt, zs, st.S1);
                st.S2 = __builtin_fmaf(wgt * zs, zs, st.S2);
                const uint32_t jpos = __float_as_uint(sm.a[1][k].z);    // run position
                if (MEDIAN && st.T > 0.5f) {         // T before this entry
                    st.zmed = e.z;
                    st.kmed = jpos + 1u;
                }
                st.last = jpos + 1u;
            };
            if (PLAIN) {
                // no per-wave bookkeeping: the lanes that do not blend skip the
                // block, and the wave skips it when none does
                if (px_live != 0u && e.pass) {
                    eval_finish(g2, g3, rc.alpha_max, e);
                    const float Tn = st.T * (1.0f - e.a);
                    if (Tn < rc.t_min) {
                        px_live = 0u;
                    } else {
                        accumulate(e.a * st.T);
                        st.T = Tn;
                    }
                }
                if (ballot64(px_live != 0u) == 0ull) {
                    wave_done = true;
                    break;
                }
                continue;
            }
            const bool done = px_live == 0u;
            if (COUNT) {
                n_reached += (uint64_t)__popcll(ballot64(!done));
                n_witer += 1;
                n_eval += done ? 0u : 1u;
            }
            bool blend = !done && e.pass;
            // no pixel of this wave takes the entry: nothing changes
            if (ballot64(blend) == 0ull) continue;
            if (COUNT) n_wblend += 1;
            eval_finish(g2, g3, rc.alpha_max, e);
            const float Tn = st.T * (1.0f - e.a);
            if (blend && Tn < rc.t_min) {
                px_live = 0u;
                blend = false;
            }
            float wgt = 0.f;
            if (blend) {
                wgt = e.a * st.T;
                accumulate(wgt);
                st.T = Tn;
                if (COUNT) n_eval_last = n_eval;
            }
            if (COUNT) n_blended += (uint64_t)__popcll(ballot64(blend));
            if (HITS) {
                const uint64_t bm = ballot64(blend);
                if (bm != 0ull) {
                    if (lane == bit) my_hits += (uint32_t)__popcll(bm);
                    if (STATS) {
                        // lane 0 holds the wave's max alpha, lane 32 its max weight
                        const uint32_t mx = wave_max2_bits(blend ? e.a : 0.f, wgt);
                        if ((lane & 31) == 0) atomicMax(&sm.st[lane == 0 ? 1 : 2][k], mx);
                    }
                }
            }
            if (ballot64(px_live != 0u) == 0ull) {
                wave_done = true;
                break;
            }
          }
          if (HITS && my_hits != 0u) atomicAdd(&sm.st[0][c * 64 + lane], my_hits);
        }
        prev_cnt = cnt;
    }
    if (HITS) {
        __syncthreads();
        flush();
    }
    if (COUNT) n_upto_last += n_eval_last;
}

// The final state of a pixel of a tile that computed nothing because the
// status word was set: every output NaN, no blended entry.
__device__ __forceinline__ void poison(PixFwd& st) {
    const float q = __builtin_nanf("");
    st.T = st.C0 = st.C1 = st.C2 = st.N0 = st.N1 = st.N2 = st.S0 = st.S1 = st.S2 = st.zref = st.zmed = q;
    st.last = st.kmed = 0u;
}

// Forward outputs of one pixel from its final state.
struct PixOut {
    float C0, C1, C2, A, D, Dist;
};

__device__ __forceinline__ PixOut pix_outputs(const PixFwd& st, const TileCtx& t) {
#pragma clang fp contract(off)
    PixOut o;
    o.C0 = st.C0 + st.T * t.bg[0];
    o.C1 = st.C1 + st.T * t.bg[1];
    o.C2 = st.C2 + st.T * t.bg[2];
    o.A = 1.0f - st.T;
    // depth = sum w z = S1 + zref S0 ; dist = 2 (S0 S2 - S1^2) with z shifted by zref
    o.D = __builtin_fmaf(st.zref, st.S0, st.S1);
    const float dd = 2.0f * (st.S0 * st.S2 - st.S1 * st.S1);
    o.Dist = (dd > 0.f || dd != dd) ? dd : 0.f;      // a NaN state stays NaN
    return o;
}

__device__ __forceinline__ void write_outputs(const PixFwd& st, const PixOut& o, const TileCtx& t,
                                              float* __restrict__ color, float* __restrict__ alpha,
                                              float* __restrict__ depth, float* __restrict__ normal,
                                              float* __restrict__ dist, float* __restrict__ T_final,
                                              uint32_t* __restrict__ n_contrib) {
    const int64_t HW = (int64_t)t.W * t.H;
    const int64_t p = (int64_t)t.iy * t.W + t.ix;
    const int64_t o1 = t.pix_off + p;
    const int64_t o3 = 3 * t.pix_off + p;
    color[o3] = o.C0;
    color[o3 + HW] = o.C1;
    color[o3 + 2 * HW] = o.C2;
    normal[o3] = st.N0;
    normal[o3 + HW] = st.N1;
    normal[o3 + 2 * HW] = st.N2;
    alpha[o1] = o.A;
    depth[o1] = o.D;
    dist[o1] = o.Dist;
    T_final[o1] = st.T;
    n_contrib[o1] = st.last;
}

template <int TW, int TH, int MODE>
__global__ void __launch_bounds__(TW * TH) SR_RASTER_OCCUPANCY
k_render_fwd(const sr_camera* __restrict__ cams, int V, int N, const float4* __restrict__ geom,
             const float4* __restrict__ app, const uint2* __restrict__ rect, const uint32_t* __restrict__ vals,
             const uint2* __restrict__ ranges,
             RasterConsts rc, float* __restrict__ color, float* __restrict__ alpha, float* __restrict__ depth,
             float* __restrict__ normal, float* __restrict__ dist, float* __restrict__ T_final,
             uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ hits, float* __restrict__ max_alpha,
             float* __restrict__ max_weight, unsigned long long* __restrict__ counts,
             float* __restrict__ median_depth, uint32_t* __restrict__ median_contrib,
             const uint32_t* __restrict__ tile_order, uint32_t* __restrict__ tile_cost) {
    constexpr int NT = TW * TH;
    __shared__ FwdSmem<NT, MODE> sm;
    __shared__ uint32_t s_cost;
    // an order entry beyond the grid leaves the workgroup idle
    if (tile_order && tile_order[blockIdx.x] >= gridDim.x) return;
    TileCtx t;
    tile_ctx<TW, TH>(cams, V, ranges, t, tile_order);
    const bool failed = status_failed(rc);
    if (failed) t.n = 0u;
    const float px = (float)t.ix + 0.5f, py = (float)t.iy + 0.5f;
    PixFwd st;
    uint64_t n_reached = 0, n_blended = 0, n_witer = 0, n_wblend = 0, n_upto = 0;
    fwd_tile<TW, NT, MODE>(t, px, py, N, geom, app, rect, vals, rc, sm, st, hits, max_alpha, max_weight, n_reached,
                           n_blended,
                       n_witer, n_wblend, n_upto);
    if (failed) poison(st);
    if (MODE & kCount) {
        // per-pixel tally of the backward's pairs: summed over the wave first
        uint64_t up = n_upto;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) up += (uint64_t)__shfl_xor((long long)up, off, 64);
        if (__lane_id() == 0) {
            atomicAdd(&counts[0], (unsigned long long)n_reached);
            atomicAdd(&counts[1], (unsigned long long)n_blended);
            atomicAdd(&counts[2], (unsigned long long)n_witer);
            atomicAdd(&counts[3], (unsigned long long)n_wblend);
            atomicAdd(&counts[4], (unsigned long long)up);
        }
    }
    if ((MODE & kShade) && t.inside) write_outputs(st, pix_outputs(st, t), t, color, alpha, depth, normal, dist,
                                                   T_final, n_contrib);
    if ((MODE & kMedian) && t.inside) {
        const int64_t o1 = t.pix_off + (int64_t)t.iy * t.W + t.ix;
        median_depth[o1] = st.zmed;
        median_contrib[o1] = st.kmed;
    }
    if (tile_cost) {
        // the tile's cost for a later launch's order: its largest n_contrib
        if (threadIdx.x == 0) s_cost = 0u;
        __syncthreads();
        if (t.inside) atomicMax(&s_cost, st.last);
        __syncthreads();
        if (threadIdx.x == 0) tile_cost[t.tile] = s_cost;
    }
}

// Per-pixel inputs of the backward.
struct PixBwd {
    uint32_t ncon, kmed;
    float T, gC0, gC1, gC2, gA, gD, gN0, gN1, gN2, gS, gMed, S0, rmean, Q, Wacc;
};

__device__ __forceinline__ void pix_bwd_init(PixBwd& pb, const TileCtx& t, float Tf, uint32_t ncon, float S0,
                                             float D, float Dist) {
#pragma clang fp contract(off)
    pb.ncon = ncon;
    pb.T = Tf;
    pb.S0 = S0;
    pb.rmean = 0.f;
    pb.Q = 0.f;
    if (S0 > 0.f) {
        pb.rmean = D / S0;
        pb.Q = Dist / (2.0f * S0);
    }
    pb.Wacc = (pb.gC0 * t.bg[0] + pb.gC1 * t.bg[1] + pb.gC2 * t.bg[2]) * Tf;
}

// Backward: per pixel, walk the tile list back to front from the last
// blended entry, recovering T_k = T_{k+1} / (1 - a_k).  With g_k the
// derivative of the loss by the blending weight w_k of entry k and
// W_k = sum_{j>k} g_j w_j (+ the background term), dL/da_k = T_k g_k -
// W_k / (1 - a_k).  Per-record gradients are summed over each wave by
// transposition (permlane swaps and DPP), over the workgroup in LDS, then
// added to grad_rec with one atomic per (tile, record, component); with
// grad_marks (the projection's tiles_touched) bit 31 of every record given a
// gradient is set.
// GEO: the loss has depth, normal or distortion terms (their upstream
// gradients are read); without them the depth path and six of the per-record
// components are identically zero and are not computed or reduced.
// HITS (without GEO): the backward also counts, per entry, the pixels that
// blend it (the forward's blend decisions, recomputed: positions below the
// pixel's last contributor that pass the cutoff), in the free component of
// the wave reduction, and adds the count to hits[g] at the flush.
template <int TW, int NT, int BATCH, bool GEO, bool HITS = false>
__device__ __forceinline__ void bwd_tile(const TileCtx& t, float px, float py, int N, const float4* __restrict__ geom,
                                         const float4* __restrict__ app, const uint32_t* __restrict__ vals,
                                         const RasterConsts& rc, BwdSmem<BATCH>& sm, PixBwd pb,
                                         float* __restrict__ grad_rec, uint32_t* __restrict__ grad_marks,
                                         uint32_t* __restrict__ hits = nullptr,
                                         uint32_t* __restrict__ cost_out = nullptr,
                                         const uint32_t* bitcache = nullptr) {
    static_assert(BATCH <= NT, "one record per thread and batch");
    static_assert(!(HITS && GEO), "the count takes a component slot of the depth terms");
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    __syncthreads();
    if (tid == 0) sm.maxn = 0u;
    __syncthreads();
    atomicMax(&sm.maxn, pb.ncon);
    __syncthreads();
    const uint32_t maxn = sm.maxn;
    // the tile's cost for the next launch's order: the run positions it works through
    if (cost_out && tid == 0) *cost_out = maxn;
    if (maxn == 0u) return;
    // entries at or beyond the wave's own last contributor concern no lane
    uint32_t wave_maxn = pb.ncon;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)wave_maxn, off, 64);
        wave_maxn = o > wave_maxn ? o : wave_maxn;
    }
    wave_maxn = __builtin_amdgcn_readfirstlane(wave_maxn);   // uniform: keep the loop control scalar
    float T = pb.T, Wacc = pb.Wacc;
    static_assert(NT / 64 <= kMaxWaves, "gathering counts");
    // batches of up to BATCH entries of the tile below run position hi,
    // gathered from its group's run highest first into slots [lo, BATCH)
    int64_t hi = maxn;
    while (hi > 0) {
        __syncthreads();
        int fill = 0;
        while (fill < BATCH && hi > 0) {
            int64_t next;
            fill += gather_round<NT, false>(t, vals, hi, fill, BATCH, sm.a[0], sm.a[1], sm.wcnt, next);
            hi = next;
        }
        const int lo = BATCH - fill;
        if (tid < BATCH) {
            if (tid >= lo) {
                const uint32_t gv = __float_as_uint(sm.a[0][tid].x);
                const uint32_t jpos = __float_as_uint(sm.a[1][tid].z);
                const size_t r = (size_t)t.v * N + (gv & kInstIdMask);
                float4 gq[kGeomF4];
#pragma unroll
                for (int q = 0; q < kGeomF4; ++q) {
                    gq[q] = geom[kGeomF4 * r + q];
                    sm.g[q][tid] = gq[q];
                }
                const float4 a0 = app[kAppF4 * r], a1 = app[kAppF4 * r + 1];
                sm.a[0][tid] = a0;
                reinterpret_cast<float2*>(&sm.a[1][tid])[0] = make_float2(a1.x, a1.y);
                // the forward's wave bits of this position when cached
                const uint32_t bits = (bitcache && jpos < BitCache<NT>::kPos)
                                          ? (bitcache[jpos >> 3] >> ((jpos & 7u) << 2)) & 0xFu
                                          : wave_bits<TW, NT / 64>(gq[0], gq[1], gq[2], gq[3].w, a1, t.tx0, t.ty0);
                // entries at or beyond the wave's last contributor concern no lane of it
                reinterpret_cast<float2*>(&sm.a[1][tid])[1] = make_float2(__uint_as_float(jpos), __uint_as_float(bits));
                sm.rec[tid] = (uint32_t)r;
            }
#pragma unroll
            for (int i = 0; i < kNumGrad; ++i) sm.acc[tid][i] = 0.f;
        }
        __syncthreads();
        // entries skipped by the forward for this wave are skipped here too
        for (int c = (BATCH - 1) >> 6; c >= (lo >> 6); --c) {
          uint64_t live = wave_live_mask_from(sm.a[1], c, lo, BATCH, wave_maxn);
          while (live != 0ull) {
            const int hb = 63 - (int)__builtin_clzll(live);
            live &= ~(1ull << hb);
            const int k = c * 64 + hb;
            const uint32_t jj = __float_as_uint(sm.a[1][k].z);    // run position
            PairEval e;
            const float4 g2 = sm.g[2][k], g3 = sm.g[3][k];
            eval_test(sm.g[0][k], sm.g[1][k], g2, g3, px, py, e);
            const bool bl = (jj < pb.ncon) && e.pass;
            if (ballot64(bl) == 0ull) continue;
            eval_finish(g2, g3, rc.alpha_max, e);
            // Gradients of this entry, branch-free: lanes that do not blend it
            // produce exact zeros (dL/da and the weight are selected to 0, the
            // intersection terms of low-pass lanes are selected away).
            const float4 a0 = sm.a[0][k], a1 = sm.a[1][k];
            const float o = g2.w;
            const float rin = __builtin_amdgcn_rcpf(1.0f - e.a);
            const float Tk = T * rin;
            const float wraw = e.a * Tk;
            const float wgt = bl ? wraw : 0.f;
            float gk = pb.gC0 * a0.x + pb.gC1 * a0.y + pb.gC2 * a0.z + pb.gA;
            float dLdz = 0.f;
            float gr[kNumGrad];
            if (GEO) {
                const float zr = e.z - pb.rmean;
                gk += pb.gD * e.z + pb.gN0 * a0.w + pb.gN1 * a1.x + pb.gN2 * a1.y +
                      pb.gS * 2.0f * (pb.Q + pb.S0 * zr * zr);
                // the median depth is the depth of entry kmed - 1 (0-based)
                const float gmed = jj + 1u == pb.kmed ? pb.gMed : 0.f;
                dLdz = bl ? __builtin_fmaf(wraw, pb.gD + 4.0f * pb.gS * pb.S0 * zr, gmed) : 0.f;
                gr[18] = pb.gN0 * wgt; gr[19] = pb.gN1 * wgt; gr[20] = pb.gN2 * wgt;
            }
            const float dLda = bl ? Tk * gk - Wacc * rin : 0.f;
            Wacc = bl ? __builtin_fmaf(gk, wraw, Wacc) : Wacc;
            T = bl ? Tk : T;
            gr[15] = pb.gC0 * wgt; gr[16] = pb.gC1 * wgt; gr[17] = pb.gC2 * wgt;
            const float dLdo = e.clamped ? 0.f : dLda * e.G;
            const float dLdG = e.clamped ? 0.f : dLda * o;
            gr[11] = dLdo;
            const float dLdrho = -e.G * dLdG;
            const float us = e.surf ? e.u : 0.f, vs = e.surf ? e.v : 0.f, rs = e.surf ? e.r : 0.f;
            float du = dLdrho * us, dv = dLdrho * vs;
            if (GEO) {
                const float dzs = e.surf ? dLdz : 0.f;
                du += dzs * g3.x;
                dv += dzs * g3.y;
                gr[12] = dzs * us; gr[13] = dzs * vs; gr[14] = dLdz;
            }
            const float dw0 = du * rs, dw1 = dv * rs;
            const float dw2 = -(du * us + dv * vs) * rs;
            gr[0] = dw0 * e.dx; gr[1] = dw1 * e.dx; gr[2] = dw2 * e.dx;
            gr[3] = dw0 * e.dy; gr[4] = dw1 * e.dy; gr[5] = dw2 * e.dy;
            gr[6] = dw0; gr[7] = dw1; gr[8] = dw2;
            const float f2 = e.surf ? 0.f : -2.0f * dLdrho;
            gr[9] = f2 * e.dx;
            gr[10] = f2 * e.dy;
            // Wave totals by transposition; the lanes holding distinct
            // components add them into the workgroup accumulator.
            {
                float c16[16];
#pragma unroll
                for (int i = 0; i < 12; ++i) c16[i] = gr[i];
                c16[12] = gr[15]; c16[13] = gr[16]; c16[14] = gr[17];
                // HITS: the blending pixels, summed exactly (at most 64 per wave)
                c16[15] = HITS && bl ? 1.f : 0.f;
                const float tot = wave_tsum<16>(c16);
                const int ci = wave_tsum_comp<16>(lane);
                // components 12..14 go to slots 15..17; the count to slot 12 (a depth slot)
                if ((lane & 12) == 0 && ci < (HITS ? 16 : 15))
                    atomicAdd(&sm.acc[k][ci < 12 ? ci : (ci < 15 ? ci + 3 : 12)], tot);
            }
            if (GEO) {
                float c8[8] = {gr[12], gr[13], gr[14], gr[18], gr[19], gr[20], 0.f, 0.f};
                const float tot = wave_tsum<8>(c8);
                const int ci = wave_tsum_comp<8>(lane);
                if ((lane & 14) == 0 && ci < 6) atomicAdd(&sm.acc[k][ci < 3 ? 12 + ci : 15 + ci], tot);
            }
          }
        }
        __syncthreads();
        if (tid >= lo && tid < BATCH) {
            float* dst = grad_rec + (size_t)sm.rec[tid] * SR_GRAD_STRIDE;
            bool any = false;
#pragma unroll
            for (int i = 0; i < kNumGrad; ++i) {
                if (HITS && i == 12) continue;
                const float vsum = sm.acc[tid][i];
                if (vsum != 0.f) {
                    atomicAdd(&dst[i], vsum);
                    any = true;
                }
            }
            // mark the record for the projection backward (bit 31)
            if (grad_marks && any) atomicOr(&grad_marks[sm.rec[tid]], 0x80000000u);
            if (HITS) {
                const uint32_t n = (uint32_t)sm.acc[tid][12];
                if (n != 0u) atomicAdd(&hits[sm.rec[tid] - (uint32_t)t.v * (uint32_t)N], n);
            }
        }
    }
}

template <int TW, int TH, int BATCH, bool GEO>
__global__ void __launch_bounds__(TW * TH) SR_RASTER_OCCUPANCY
k_render_bwd(const sr_camera* __restrict__ cams, int V, int N, const float4* __restrict__ geom,
             const float4* __restrict__ app, const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
             RasterConsts rc, const float* __restrict__ alpha, const float* __restrict__ depth,
             const float* __restrict__ dist, const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
             const float* __restrict__ dC, const float* __restrict__ dA, const float* __restrict__ dD,
             const float* __restrict__ dNrm, const float* __restrict__ dDist,
             const uint32_t* __restrict__ median_contrib, const float* __restrict__ dMed,
             float* __restrict__ grad_rec, uint32_t* __restrict__ grad_marks,
             const uint32_t* __restrict__ tile_order) {
    __shared__ BwdSmem<BATCH> sm;
    // an order entry beyond the grid leaves the workgroup idle; so does a set
    // status word (no gradients)
    if (tile_order && tile_order[blockIdx.x] >= gridDim.x) return;
    if (status_failed(rc)) return;
    TileCtx t;
    tile_ctx<TW, TH>(cams, V, ranges, t, tile_order);
    const float px = (float)t.ix + 0.5f, py = (float)t.iy + 0.5f;
    PixBwd pb;
    pb.gC0 = pb.gC1 = pb.gC2 = pb.gA = pb.gD = pb.gN0 = pb.gN1 = pb.gN2 = pb.gS = pb.gMed = 0.f;
    pb.ncon = pb.kmed = 0;
    pb.T = 1.f;
    pb.S0 = pb.rmean = pb.Q = pb.Wacc = 0.f;
    if (t.inside) {
        const int64_t HW = (int64_t)t.W * t.H;
        const int64_t p = (int64_t)t.iy * t.W + t.ix;
        const int64_t o1 = t.pix_off + p, o3 = 3 * t.pix_off + p;
        if (dC) { pb.gC0 = dC[o3]; pb.gC1 = dC[o3 + HW]; pb.gC2 = dC[o3 + 2 * HW]; }
        if (dA) pb.gA = dA[o1];
        if (dD) pb.gD = dD[o1];
        if (dNrm) { pb.gN0 = dNrm[o3]; pb.gN1 = dNrm[o3 + HW]; pb.gN2 = dNrm[o3 + 2 * HW]; }
        if (dDist) pb.gS = dDist[o1];
        if (dMed) { pb.gMed = dMed[o1]; pb.kmed = median_contrib[o1]; }
        pix_bwd_init(pb, t, T_final[o1], n_contrib[o1], alpha[o1], depth[o1], dist[o1]);
    }
    bwd_tile<TW, TW * TH, BATCH, GEO>(t, px, py, N, geom, app, vals, rc, sm, pb, grad_rec, grad_marks);
}

// One training step of the compositing for a tile: forward, the masked L1 +
// background loss gradients of every pixel (Eq. 1, Eq. 2) and the backward,
// with the per-pixel state kept in registers between the phases.  STATS = 1
// counts the blended pixels of every surfel (the usage record of Section
// 4.3), taken by the backward, which recomputes the same blend decisions;
// STATS = 2 has the forward take the count and the maximum alpha and weight;
// 0 records nothing.  Per-tile loss partial sums go to tile_loss[2*tile]
// (L_b numerator, L1 numerator).
template <int TW, int TH, int BATCH, int STATS>
__global__ void __launch_bounds__(TW * TH) SR_RASTER_OCCUPANCY
k_train_raster(const sr_camera* __restrict__ cams, int V, int N, const float4* __restrict__ geom,
               const float4* __restrict__ app, const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
               RasterConsts rc, const uint8_t* __restrict__ mask, const float* __restrict__ target, float gamma,
               float w_c, float* __restrict__ color, float* __restrict__ alpha, float* __restrict__ depth,
               float* __restrict__ normal, float* __restrict__ dist, float* __restrict__ T_final,
               uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ hits, float* __restrict__ max_alpha,
               float* __restrict__ max_weight, float* __restrict__ tile_loss, float* __restrict__ grad_rec,
               uint32_t* __restrict__ grad_marks,
               const uint32_t* __restrict__ tile_order, uint32_t* __restrict__ tile_cost) {
    constexpr int NT = TW * TH;
    constexpr int MODE = kShade | (STATS == 2 ? kStats : 0);
    constexpr size_t kF = sizeof(FwdSmem<NT, MODE>), kB = sizeof(BwdSmem<BATCH>);
    __shared__ __align__(16) unsigned char smem[kF > kB ? kF : kB];
    __shared__ float s_red[NT];
    // the wave-bit cache, except with the full statistics (whose larger
    // forward staging would lose a workgroup per CU to the extra LDS)
    constexpr bool CACHE = STATS != 2;
    __shared__ uint32_t s_bits[CACHE ? BitCache<NT>::kWords : 1];
    TileCtx t;
    // an order entry beyond the grid leaves the workgroup idle (not a valid
    // permutation: nothing of it is written)
    if (tile_order && tile_order[blockIdx.x] >= gridDim.x) return;
    tile_ctx<TW, TH>(cams, V, ranges, t, tile_order);
    // a set status word: nothing blended, NaN outputs and losses, no gradients
    const bool failed = status_failed(rc);
    if (failed) t.n = 0u;
    const float px = (float)t.ix + 0.5f, py = (float)t.iy + 0.5f;
    PixFwd st;
    uint64_t n0 = 0, n1 = 0, n2 = 0, n3 = 0, n4 = 0;
    if (CACHE) {
        for (int i = threadIdx.x; i < BitCache<NT>::kWords; i += NT) s_bits[i] = 0u;
        __syncthreads();
    }
    fwd_tile<TW, NT, MODE>(t, px, py, N, geom, app, nullptr, vals, rc, *reinterpret_cast<FwdSmem<NT, MODE>*>(smem), st,
                           hits, max_alpha, max_weight, n0, n1, n2, n3, n4, CACHE ? s_bits : nullptr);
    if (failed) poison(st);
    const PixOut o = pix_outputs(st, t);
    PixBwd pb;
    pb.gC0 = pb.gC1 = pb.gC2 = pb.gA = pb.gD = pb.gN0 = pb.gN1 = pb.gN2 = pb.gS = pb.gMed = 0.f;
    pb.ncon = pb.kmed = 0;
    pb.T = 1.f;
    pb.S0 = pb.rmean = pb.Q = pb.Wacc = 0.f;
    float lb = 0.f, l1 = 0.f;
    if (t.inside) {
        write_outputs(st, o, t, color, alpha, depth, normal, dist, T_final, n_contrib);
        // the same per-pixel loss terms and gradients as sr_background_loss
        const int64_t HW = (int64_t)t.W * t.H;
        const int64_t p = (int64_t)t.iy * t.W + t.ix;
        const int64_t o1 = t.pix_off + p, o3 = 3 * t.pix_off + p;
        const float Cv[3] = {o.C0, o.C1, o.C2};
        const float Iv[3] = {target[o3], target[o3 + HW], target[o3 + 2 * HW]};
        float gC[3];
        pixel_loss_grad(mask[o1], o.A, Cv, Iv, gamma, w_c, (float)HW, (float)V, lb, l1, pb.gA, gC);
        pb.gC0 = gC[0]; pb.gC1 = gC[1]; pb.gC2 = gC[2];
        pix_bwd_init(pb, t, st.T, st.last, o.A, o.D, o.Dist);
    }
    // per-tile loss partials, fixed-order tree
    __syncthreads();
    s_red[threadIdx.x] = lb;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_loss[2 * (size_t)t.tile] = s_red[0];
    __syncthreads();
    s_red[threadIdx.x] = l1;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_loss[2 * (size_t)t.tile + 1] = s_red[0];
    bwd_tile<TW, NT, BATCH, false, STATS == 1>(t, px, py, N, geom, app, vals, rc,
                                               *reinterpret_cast<BwdSmem<BATCH>*>(smem), pb, grad_rec, grad_marks, hits,
                                               tile_cost ? tile_cost + t.tile : nullptr, CACHE ? s_bits : nullptr);
}

__global__ void k_fill_f32(float* __restrict__ p, float v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// A set status word (statistics incomplete) prunes nothing.
__global__ void k_prune_mask(int N, const float* __restrict__ max_alpha, float tau, const uint32_t* __restrict__ status,
                             uint8_t* __restrict__ mask) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool failed = status != nullptr && *status != 0u;
    if (g < N) mask[g] = (!failed && max_alpha[g] < tau) ? 1 : 0;
}

// Records per LDS batch of the backward: compiled for 32, 64, 128 and 256,
// each at most the tile's pixel count (one staging thread per record).  The
// default, min(128, pixels), keeps the separate backward's LDS footprint and
// hence its occupancy in check; in the fused kernel the forward's staging
// area is as large, so only 256 costs occupancy there.
constexpr int kBwdBatch = 128;

constexpr int resolve_batch(int pixels, int batch) {
    return batch != 0 ? batch : (pixels < kBwdBatch ? pixels : kBwdBatch);
}

// Calls f(integral_constant<int, B>) for the compiled batch B == batch (a
// value of resolve_batch); false when it is not compiled for this tile.
template <int PIX, typename F>
bool with_batch(int batch, F&& f) {
    switch (batch) {
        case 32: if constexpr (32 <= PIX) { f(std::integral_constant<int, 32>{}); return true; } break;
        case 64: if constexpr (64 <= PIX) { f(std::integral_constant<int, 64>{}); return true; } break;
        case 128: if constexpr (128 <= PIX) { f(std::integral_constant<int, 128>{}); return true; } break;
        case 256: if constexpr (256 <= PIX) { f(std::integral_constant<int, 256>{}); return true; } break;
        default: break;
    }
    return false;
}

template <int TW, int TH, int MODE>
void fwd_launch(int total_tiles, hipStream_t s, const sr_camera* cams, int V, int N, const float4* geom,
                const float4* app, const uint2* rect, const uint32_t* vals, const uint2* ranges, RasterConsts rc,
                float* color,
                float* alpha, float* depth, float* normal, float* dist, float* T_final, uint32_t* n_contrib,
                uint32_t* hits, float* max_alpha, float* max_weight, unsigned long long* counts,
                float* median_depth, uint32_t* median_contrib, const uint32_t* tile_order, uint32_t* tile_cost) {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, MODE>), dim3(total_tiles), dim3(TW * TH), 0, s, cams, V, N, geom, app,
                       rect, vals, ranges, rc, color, alpha, depth, normal, dist, T_final, n_contrib, hits, max_alpha,
                       max_weight, counts, median_depth, median_contrib, tile_order, tile_cost);
}

template <int TW, int TH>
bool fwd_dispatch(int mode, int total_tiles, hipStream_t s, const sr_camera* cams, int V, int N,
                  const float4* geom, const float4* app, const uint2* rect, const uint32_t* vals, const uint2* ranges,
                  RasterConsts rc, float* color, float* alpha, float* depth, float* normal, float* dist,
                  float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha, float* max_weight,
                  unsigned long long* counts, float* median_depth, uint32_t* median_contrib,
                  const uint32_t* tile_order, uint32_t* tile_cost) {
#define SR_FWD(M)                                                                                        \
    fwd_launch<TW, TH, M>(total_tiles, s, cams, V, N, geom, app, rect, vals, ranges, rc, color, alpha, depth, \
                          normal, dist, T_final, n_contrib, hits, max_alpha, max_weight, counts,          \
                          median_depth, median_contrib, tile_order, tile_cost)
    switch (mode) {
        case kShade: SR_FWD(kShade); return true;
        case kShade | kHits: SR_FWD(kShade | kHits); return true;
        case kShade | kStats: SR_FWD(kShade | kStats); return true;
        case kShade | kMedian: SR_FWD(kShade | kMedian); return true;
        case kShade | kHits | kMedian: SR_FWD(kShade | kHits | kMedian); return true;
        case kShade | kStats | kMedian: SR_FWD(kShade | kStats | kMedian); return true;
        case kStats: SR_FWD(kStats); return true;
        case kStats | kRect: SR_FWD(kStats | kRect); return true;
        case kCount: SR_FWD(kCount); return true;
        default: return false;       // not compiled
    }
#undef SR_FWD
}

template <int TW, int TH>
bool bwd_launch(int batch, int total_tiles, hipStream_t s, const sr_camera* cams, int V, int N, const float4* geom,
                const float4* app, const uint32_t* vals, const uint2* ranges, RasterConsts rc, const float* alpha,
                const float* depth, const float* dist, const float* T_final, const uint32_t* n_contrib,
                const float* dC, const float* dA, const float* dD, const float* dN, const float* dS,
                const uint32_t* median_contrib, const float* dMed, float* grad_rec, uint32_t* grad_marks,
                const uint32_t* tile_order) {
    const bool geo = dD || dN || dS || dMed;
    return with_batch<TW * TH>(resolve_batch(TW * TH, batch), [&](auto bc) {
        constexpr int B = decltype(bc)::value;
        if (geo)
            hipLaunchKernelGGL((k_render_bwd<TW, TH, B, true>), dim3(total_tiles), dim3(TW * TH), 0, s, cams, V, N,
                               geom, app, vals, ranges, rc, alpha, depth, dist, T_final, n_contrib, dC, dA, dD, dN,
                               dS, median_contrib, dMed, grad_rec, grad_marks, tile_order);
        else
            hipLaunchKernelGGL((k_render_bwd<TW, TH, B, false>), dim3(total_tiles), dim3(TW * TH), 0, s, cams, V, N,
                               geom, app, vals, ranges, rc, alpha, depth, dist, T_final, n_contrib, dC, dA, dD, dN,
                               dS, median_contrib, dMed, grad_rec, grad_marks, tile_order);
    });
}

template <int TW, int TH>
bool train_launch(int stats, int batch, int total_tiles, hipStream_t s, const sr_camera* cams, int V, int N,
                  const float4* geom, const float4* app, const uint32_t* vals, const uint2* ranges, RasterConsts rc,
                  const uint8_t* mask, const float* target, float gamma, float w_c, float* color, float* alpha,
                  float* depth, float* normal, float* dist, float* T_final, uint32_t* n_contrib, uint32_t* hits,
                  float* max_alpha, float* max_weight, float* tile_loss, float* grad_rec, uint32_t* grad_marks,
                  const uint32_t* tile_order,
                  uint32_t* tile_cost) {
    return with_batch<TW * TH>(resolve_batch(TW * TH, batch), [&](auto bc) {
        constexpr int B = decltype(bc)::value;
#define SR_TRAIN(S)                                                                                              \
    hipLaunchKernelGGL((k_train_raster<TW, TH, B, S>), dim3(total_tiles), dim3(TW * TH), 0, s, cams, V, N, geom, \
                       app, vals, ranges, rc, mask, target, gamma, w_c, color, alpha, depth, normal, dist, T_final, \
                       n_contrib, hits, max_alpha, max_weight, tile_loss, grad_rec, grad_marks, tile_order, tile_cost)
        if (stats == 2)
            SR_TRAIN(2);
        else if (stats == 1)
            SR_TRAIN(1);
        else
            SR_TRAIN(0);
#undef SR_TRAIN
    });
}

// Compiled tile shapes (the binning takes any shape; the raster kernels are
// instantiated for these).
#define SR_TILE_SHAPES(X) X(16, 16) X(16, 8) X(8, 8) X(32, 8)

}  // namespace

bool tile_shape_supported(int tw, int th) {
#define SR_TS(W, H) if (tw == W && th == H) return true;
    SR_TILE_SHAPES(SR_TS)
#undef SR_TS
    return false;
}

bool bwd_batch_supported(int tw, int th, int batch) {
    if (!tile_shape_supported(tw, th)) return false;
    const int b = resolve_batch(tw * th, batch);
    return (b == 32 || b == 64 || b == 128 || b == 256) && b <= tw * th;
}

hipError_t fill_f32(float* p, float v, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_render_fwd(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                             const float* geom, const float* app, const uint16_t* rect, const uint32_t* vals,
                             const uint32_t* ranges, float* color, float* alpha, float* depth, float* normal,
                             float* dist, float* T_final, uint32_t* n_contrib, uint32_t* hits, float* max_alpha,
                             float* max_weight, unsigned long long* counts, float* median_depth,
                             uint32_t* median_contrib, const uint32_t* tile_order, uint32_t* tile_cost,
                             const uint32_t* status, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    RasterConsts rc{cfg.alpha_min, cfg.alpha_max, cfg.t_min, cfg.flags, status};
    const int stats = hits ? (max_alpha ? kStats : kHits) : 0;
    int mode = counts ? kCount
                      : ((color ? kShade : 0) | stats | (color && median_depth ? kMedian : 0) |
                         (!color && hits && rect ? kRect : 0));
#define SR_TS(W, H)                                                                                              \
    if (cfg.tile_w == W && cfg.tile_h == H) {                                                                   \
        if (!fwd_dispatch<W, H>(mode, total_tiles, s, cams, V, N, (const float4*)geom, (const float4*)app,     \
                                (const uint2*)rect, vals, (const uint2*)ranges, rc, color, alpha, depth, normal, \
                                dist, T_final, n_contrib, hits, max_alpha, max_weight, counts, median_depth,     \
                                median_contrib, tile_order, tile_cost))                                         \
            return hipErrorInvalidValue;                                                                        \
        return hipGetLastError();                                                                               \
    }
    SR_TILE_SHAPES(SR_TS)
#undef SR_TS
    return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                             const float* geom, const float* app, const uint32_t* vals, const uint32_t* ranges,
                             const float* alpha, const float* depth, const float* dist, const float* T_final,
                             const uint32_t* n_contrib, const float* dC, const float* dA, const float* dD,
                             const float* dN, const float* dS, const uint32_t* median_contrib, const float* dMed,
                             float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order,
                             const uint32_t* status, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    RasterConsts rc{cfg.alpha_min, cfg.alpha_max, cfg.t_min, cfg.flags, status};
#define SR_TS(W, H)                                                                                            \
    if (cfg.tile_w == W && cfg.tile_h == H) {                                                                 \
        if (!bwd_launch<W, H>(cfg.bwd_batch, total_tiles, s, cams, V, N, (const float4*)geom,                 \
                              (const float4*)app, vals, (const uint2*)ranges, rc, alpha, depth, dist, T_final,  \
                              n_contrib, dC, dA, dD, dN, dS, median_contrib, dMed, grad_rec, grad_marks,       \
                              tile_order))                                                                      \
            return hipErrorInvalidValue;                                                                      \
        return hipGetLastError();                                                                             \
    }
    SR_TILE_SHAPES(SR_TS)
#undef SR_TS
    return hipErrorInvalidValue;
}

hipError_t launch_train_raster(const sr_config& cfg, int N, int V, int total_tiles, const sr_camera* cams,
                               const float* geom, const float* app, const uint32_t* vals, const uint32_t* ranges,
                               const uint8_t* mask, const float* target, float gamma, float w_c, float* color,
                               float* alpha, float* depth, float* normal, float* dist, float* T_final,
                               uint32_t* n_contrib, uint32_t* hits, float* max_alpha, float* max_weight,
                               float* tile_loss, float* grad_rec, uint32_t* grad_marks, const uint32_t* tile_order,
                               uint32_t* tile_cost,
                               const uint32_t* status, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    RasterConsts rc{cfg.alpha_min, cfg.alpha_max, cfg.t_min, cfg.flags, status};
#define SR_TS(W, H)                                                                                               \
    if (cfg.tile_w == W && cfg.tile_h == H) {                                                                    \
        if (!train_launch<W, H>(hits ? (max_alpha ? 2 : 1) : 0, cfg.bwd_batch, total_tiles, s, cams, V, N,      \
                                (const float4*)geom, (const float4*)app, vals, (const uint2*)ranges, rc, mask,   \
                                target, gamma, w_c, color, alpha, depth, normal, dist, T_final, n_contrib, hits, \
                                max_alpha, max_weight, tile_loss, grad_rec, grad_marks, tile_order, tile_cost)) \
            return hipErrorInvalidValue;                                                                         \
        return hipGetLastError();                                                                                \
    }
    SR_TILE_SHAPES(SR_TS)
#undef SR_TS
    return hipErrorInvalidValue;
}

// ---- the allocation-free training step ------------------------------------------
//
// The per-tile loss partials of sr_train_step_raster_noalloc live in this
// file-scope device array (one copy per GPU, held until the process ends)
// instead of a caller buffer.  On the host its name is a stand-in symbol, not
// a device address: host code uses only the address hipGetSymbolAddress
// returns, taken once per device with that device current.
__device__ __align__(256) float scratch[2 * SR_NOALLOC_MAX_TILES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, float** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[device] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

hipError_t launch_prune_mask(int N, const float* max_alpha, float tau, const uint32_t* status, uint8_t* mask,
                             hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prune_mask, dim3((N + 255) / 256), dim3(256), 0, s, N, max_alpha, tau, status, mask);
    return hipGetLastError();
}

}  // namespace sr
