// Duplicate-key generation, sorting and per-tile ranges.
//
// Section 4.3: each pixel blends the Gaussians assigned to it in
// front-to-back order.  The assignment is materialised as instances
// (view, tile group, surfel) sorted by the 64-bit key (global group id << 32
// | float32 depth bits), ties by surfel id, where a group is 4 x 4 tiles:
// one instance per group the surfel's tile rectangle meets, carrying the
// part of the rectangle inside the group, so a tile reads its group's run
// and keeps the entries that cover it.  Grouping cuts the instances (and the
// sort) several-fold; the tiles' lists are unchanged.
//
// An LSD radix sort of that key processes the depth digits first and the
// group digits last.  The depth of an instance is the depth of its surfel,
// so the depth passes run once over the visible (view, surfel) pairs before
// duplication instead of over the instances; the instances are then emitted
// in depth order and only the ceil(log2(groups)) group bits are sorted, by a
// stable LSD radix sort.
// Every count lives in device memory, so the sequence needs no host
// synchronisation and can be captured into a HIP graph.
#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr int kNT = 256;            // threads per block
constexpr int kTile = kNT * 32;     // block chunks are multiples of the largest radix sub-tile
constexpr int kMaxDigitBits = 9;    // radix digits of up to 9 bits (512 buckets)
constexpr int kMaxRadix = 1 << kMaxDigitBits;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan over the 256 threads of a block; total returned in *total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave /*[4]*/, T* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    T incl = wave_incl_scan(v);
    if (lane == 63) s_wave[w] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kNT / 64; ++i) {
        T s = s_wave[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__device__ __forceinline__ void static_chunk(uint64_t n, int G, uint64_t* begin, uint64_t* end) {
    uint64_t chunk = (n + G - 1) / G;
    chunk = (chunk + kNT - 1) / kNT * kNT;
    *begin = (uint64_t)blockIdx.x * chunk;
    uint64_t e = *begin + chunk;
    *end = e < n ? e : n;
}

__device__ __forceinline__ void radix_chunk(uint32_t n, int G, uint32_t* begin, uint32_t* end) {
    uint32_t chunk = (n + G - 1) / G;
    chunk = (chunk + kTile - 1) / kTile * kTile;
    uint64_t b = (uint64_t)blockIdx.x * chunk;
    uint64_t e = b + chunk;
    *begin = (uint32_t)(b < n ? b : n);
    *end = (uint32_t)(e < n ? e : n);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---- visible (view, surfel) pairs -------------------------------------------

__global__ void __launch_bounds__(kNT)
k_vis_count(uint64_t VN, int G, const uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ sums) {
    __shared__ uint32_t s_w[4];
    uint64_t b, e;
    static_chunk(VN, G, &b, &e);
    uint32_t c = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += kNT) c += tiles_touched[i] > 0u ? 1u : 0u;
    uint32_t tot;
    block_excl_scan<uint32_t>(c, s_w, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of n (<= 4096) block sums in place; total to *out
template <typename T>
__global__ void __launch_bounds__(kNT)
k_scan_small(T* __restrict__ data, int n, uint32_t* __restrict__ counters, int slot, uint32_t capacity,
             uint64_t* __restrict__ total64, uint32_t* __restrict__ status = nullptr) {
    __shared__ T s_w[4];
    const int per = (n + kNT - 1) / kNT;
    const int b = threadIdx.x * per;
    T loc[16];
    T sum = 0;
    for (int i = 0; i < per; ++i) {
        loc[i] = (b + i < n) ? data[b + i] : 0;
        sum += loc[i];
    }
    T tot;
    T run = block_excl_scan<T>(sum, s_w, &tot);
    for (int i = 0; i < per; ++i) {
        if (b + i < n) data[b + i] = run;
        run += loc[i];
    }
    if (threadIdx.x == 0) {
        if (slot == 0) {
            counters[0] = (uint32_t)tot;
        } else {
            const uint64_t t64 = (uint64_t)tot;
            *total64 = t64;
            counters[1] = t64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t64;
            counters[2] = t64 > capacity ? capacity : (uint32_t)t64;
            counters[3] = t64 > capacity ? 1u : 0u;
            if (t64 > capacity && status) {
                // sticky until the caller clears it: later compositing calls
                // of the context see truncated lists and flag their outputs
                atomicOr(&status[0], (uint32_t)SR_STATUS_CAPACITY);
                atomicMax(&status[1], counters[1]);
            }
        }
    }
}

__global__ void __launch_bounds__(kNT)
k_vis_compact(uint64_t VN, int G, const uint32_t* __restrict__ tiles_touched,
              const uint32_t* __restrict__ depth_key, const uint32_t* __restrict__ offs,
              uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_w[4];
    uint64_t b, e;
    static_chunk(VN, G, &b, &e);
    uint32_t run = offs[blockIdx.x];
    for (uint64_t base = b; base < e; base += kNT) {
        const uint64_t i = base + threadIdx.x;
        const bool vis = i < e && tiles_touched[i] > 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<uint32_t>(vis ? 1u : 0u, s_w, &tot);
        if (vis) {
            keys[run + ex] = depth_key[i];
            vals[run + ex] = (uint32_t)i;
        }
        run += tot;
    }
}

// ---- stable LSD radix sort of (u32 key, u32 value), count in device memory --

__global__ void __launch_bounds__(kNT)
k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ count, int G, int shift, int bits,
             uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[4][kMaxRadix];
    const int R = 1 << bits, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * kMaxRadix; i += kNT) (&s_h[0][0])[i] = 0;
    __syncthreads();
    uint32_t b, e;
    radix_chunk(*count, G, &b, &e);
    const uint32_t mask = (uint32_t)R - 1u;
    const int lane = __lane_id();
    // eight independent loads in flight per thread; a digit held by many
    // lanes of the wave (skewed digits: the top byte of positive depths, the
    // high bits of group ids) is added once for all of them instead of by
    // every lane into the same LDS word
    uint32_t i = b + threadIdx.x;
    for (; i + 7u * kNT < e; i += 8u * kNT) {
        uint32_t k[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) k[u] = keys[i + (uint32_t)u * kNT];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            // d0: the digit of the wave's first active lane (the loop bound
            // depends on the thread, so lane 0 may have left at a chunk's end)
            const uint32_t d = (k[u] >> shift) & mask;
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
            const int leader = __builtin_amdgcn_readfirstlane(lane);
            const uint64_t same = __ballot(d == d0);
            const int n0 = __popcll(same);
            if (n0 >= 16) {
                if (lane == leader) atomicAdd(&s_h[w][d0], (uint32_t)n0);
                if (d != d0) atomicAdd(&s_h[w][d], 1u);
            } else {
                atomicAdd(&s_h[w][d], 1u);
            }
        }
    }
    for (; i < e; i += kNT) atomicAdd(&s_h[w][(keys[i] >> shift) & mask], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += kNT)
        hist[(size_t)d * G + blockIdx.x] = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
}

// one block per digit: exclusive scan over the G blocks; digit total to tot[d]
__global__ void __launch_bounds__(kNT)
k_radix_digit_scan(uint32_t* __restrict__ hist, int G, uint32_t* __restrict__ tot) {
    __shared__ uint32_t s_w[4];
    uint32_t* h = hist + (size_t)blockIdx.x * G;
    const int per = (G + kNT - 1) / kNT;
    const int b = threadIdx.x * per;
    uint32_t loc[16], sum = 0;
    for (int i = 0; i < per; ++i) {
        loc[i] = (b + i < G) ? h[b + i] : 0u;
        sum += loc[i];
    }
    uint32_t total;
    uint32_t run = block_excl_scan<uint32_t>(sum, s_w, &total);
    for (int i = 0; i < per; ++i) {
        if (b + i < G) h[b + i] = run;
        run += loc[i];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Every thread owns the two digits 2*tid and 2*tid + 1 of the per-digit
// bookkeeping (up to 512 digits).
template <int IPT>
__global__ void __launch_bounds__(kNT)
k_radix_scatter(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
                const uint32_t* __restrict__ count, int G, int shift, int bits,
                const uint32_t* __restrict__ hist, const uint32_t* __restrict__ tot,
                uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
    __shared__ uint32_t s_off[kMaxRadix];
    __shared__ uint32_t s_wcnt[4][kMaxRadix];
    __shared__ uint32_t s_lstart[kMaxRadix];
    __shared__ uint32_t s_keys[kNT * IPT];
    __shared__ uint32_t s_vals[kNT * IPT];
    __shared__ uint32_t s_w[4];
    const int R = 1 << bits;
    const uint32_t mask = (uint32_t)R - 1u;
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int d0 = 2 * tid, d1 = 2 * tid + 1;
    uint32_t b, e;
    radix_chunk(*count, G, &b, &e);
    // global start of every digit for this block
    {
        const uint32_t t0 = d0 < R ? tot[d0] : 0u, t1 = d1 < R ? tot[d1] : 0u;
        uint32_t all;
        const uint32_t ex = block_excl_scan<uint32_t>(t0 + t1, s_w, &all);
        s_off[d0] = d0 < R ? ex + hist[(size_t)d0 * G + blockIdx.x] : 0u;
        s_off[d1] = d1 < R ? ex + t0 + hist[(size_t)d1 * G + blockIdx.x] : 0u;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t tb = b; tb < e; tb += kNT * IPT) {
        for (int i = tid; i < 4 * kMaxRadix; i += kNT) (&s_wcnt[0][0])[i] = 0u;
        __syncthreads();
        uint32_t kk[IPT], vv[IPT], rank[IPT];
        int dg[IPT];
        bool ok[IPT];
        const uint32_t seg = tb + (uint32_t)w * 64u * IPT;
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t idx = seg + (uint32_t)r * 64u + (uint32_t)lane;
            ok[r] = idx < e;
            kk[r] = ok[r] ? keys_in[idx] : 0u;
            vv[r] = ok[r] ? (vals_in ? vals_in[idx] : idx) : 0u;
            dg[r] = (int)((kk[r] >> shift) & mask);
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            uint64_t peers = ballot64(ok[r]);
            for (int bit = 0; bit < bits; ++bit) {
                const bool set = (dg[r] >> bit) & 1;
                const uint64_t bb = ballot64(set);
                peers &= set ? bb : ~bb;
            }
            const uint32_t before = (uint32_t)__popcll(peers & lt);
            const uint32_t cnt = (uint32_t)__popcll(peers);
            uint32_t old = ok[r] ? s_wcnt[w][dg[r]] : 0u;
            if (ok[r] && before == 0u) s_wcnt[w][dg[r]] = old + cnt;
            rank[r] = old + before;
        }
        __syncthreads();
        uint32_t dt0, dt1;
        {
            uint32_t c[2][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) { c[0][q] = s_wcnt[q][d0]; c[1][q] = s_wcnt[q][d1]; }
            dt0 = c[0][0] + c[0][1] + c[0][2] + c[0][3];
            dt1 = c[1][0] + c[1][1] + c[1][2] + c[1][3];
            uint32_t all;
            const uint32_t ls = block_excl_scan<uint32_t>(dt0 + dt1, s_w, &all);
            s_lstart[d0] = ls;
            s_lstart[d1] = ls + dt0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int d = h ? d1 : d0;
                s_wcnt[0][d] = 0u;
                s_wcnt[1][d] = c[h][0];
                s_wcnt[2][d] = c[h][0] + c[h][1];
                s_wcnt[3][d] = c[h][0] + c[h][1] + c[h][2];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            if (ok[r]) {
                const uint32_t lp = s_lstart[dg[r]] + s_wcnt[w][dg[r]] + rank[r];
                s_keys[lp] = kk[r];
                s_vals[lp] = vv[r];
            }
        }
        __syncthreads();
        const uint32_t cntTile = (e - tb) < (uint32_t)(kNT * IPT) ? (e - tb) : (uint32_t)(kNT * IPT);
        for (uint32_t i = tid; i < cntTile; i += kNT) {
            const uint32_t key = s_keys[i];
            const int d = (int)((key >> shift) & mask);
            const uint32_t dst = s_off[d] + (i - s_lstart[d]);
            if (keys_out) keys_out[dst] = key;
            vals_out[dst] = s_vals[i];
        }
        __syncthreads();
        s_off[d0] += dt0;
        s_off[d1] += dt1;
        __syncthreads();
    }
}

// ---- instances ----------------------------------------------------------------

// Tile groups met by the rectangle of a record; a group spans
// 2^gsx x 2^gsy pixels (tile sides are powers of two).
__device__ __forceinline__ uint32_t groups_of(const ushort4 rc, int gsx, int gsy) {
    const int gx0 = rc.x >> gsx, gx1 = rc.y >> gsx, gy0 = rc.z >> gsy, gy1 = rc.w >> gsy;
    return (uint32_t)((gx1 - gx0 + 1) * (gy1 - gy0 + 1));
}

// Groups met by every depth-sorted visible pair and their sum per block;
// the pairs' rectangles are gathered once into depth order for the emission.
// The gather is random over the rectangle array: four independent gathers
// per thread are kept in flight.
__global__ void __launch_bounds__(kNT)
k_inst_count(const uint32_t* __restrict__ counters, int G, const uint32_t* __restrict__ vis_vals,
             const ushort4* __restrict__ rect, int gsx, int gsy, uint32_t* __restrict__ tt_sorted,
             ushort4* __restrict__ rect_sorted, uint64_t* __restrict__ sums) {
    __shared__ uint64_t s_w[4];
    constexpr int U = 4;
    uint64_t b, e;
    static_chunk(counters[0], G, &b, &e);
    uint64_t c = 0;
    uint64_t i = b + threadIdx.x;
    for (; i + (uint64_t)(U - 1) * kNT < e; i += (uint64_t)U * kNT) {
        uint32_t r[U];
        ushort4 rc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = vis_vals[i + (uint64_t)u * kNT];
#pragma unroll
        for (int u = 0; u < U; ++u) rc[u] = rect[r[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t t = groups_of(rc[u], gsx, gsy);
            tt_sorted[i + (uint64_t)u * kNT] = t;
            rect_sorted[i + (uint64_t)u * kNT] = rc[u];
            c += t;
        }
    }
    for (; i < e; i += kNT) {
        const ushort4 rc = rect[vis_vals[i]];
        const uint32_t t = groups_of(rc, gsx, gsy);
        tt_sorted[i] = t;
        rect_sorted[i] = rc;
        c += t;
    }
    uint64_t tot;
    block_excl_scan<uint64_t>(c, s_w, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive instance offset of every depth-sorted visible pair.
__global__ void __launch_bounds__(kNT)
k_inst_offsets(const uint32_t* __restrict__ counters, int G, const uint32_t* __restrict__ tt_sorted,
               const uint64_t* __restrict__ block_offs, uint64_t* __restrict__ offs) {
    __shared__ uint64_t s_w[4];
    uint64_t b, e;
    static_chunk(counters[0], G, &b, &e);
    uint64_t run = block_offs[blockIdx.x];
    for (uint64_t base = b; base < e; base += kNT) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t t = i < e ? (uint64_t)tt_sorted[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_excl_scan<uint64_t>(t, s_w, &tot);
        if (i < e) offs[i] = run + ex;
        run += tot;
    }
}

constexpr int kEmitPerBlock = 4096;   // instances written per block

// First visible pair of every emission block: the last pair whose first
// instance is at or before the block's first output position (one thread per
// block, binary search over the instance offsets).
__global__ void __launch_bounds__(kNT)
k_emit_starts(const uint32_t* __restrict__ counters, const uint64_t* __restrict__ offs, uint32_t blocks,
              uint32_t* __restrict__ starts) {
    const uint32_t b = blockIdx.x * kNT + threadIdx.x;
    if (b >= blocks) return;
    const uint32_t n_vis = counters[0];
    const uint64_t ob = (uint64_t)b * kEmitPerBlock;
    uint32_t lo = 0, hi = n_vis == 0 ? 0 : n_vis - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= ob) lo = mid; else hi = mid - 1;
    }
    starts[b] = lo;
}

// Emits the instances in depth order.  The output space is partitioned:
// block b writes instances [b*4096, (b+1)*4096), whatever the number of
// surfels they come from, so surfels covering thousands of tiles (close to
// a camera, first in depth order) do not serialise on a few blocks.
__global__ void __launch_bounds__(kNT)
k_emit(const uint32_t* __restrict__ counters, const uint64_t* __restrict__ total64, int N, int tsx, int tsy,
       const sr_camera* __restrict__ cams, const uint32_t* __restrict__ vis_vals,
       const ushort4* __restrict__ rect_sorted,
       const uint64_t* __restrict__ offs, const uint32_t* __restrict__ starts, uint32_t* __restrict__ inst_keys,
       uint32_t* __restrict__ inst_vals) {
    constexpr int GS = SR_TILE_GROUP;
    __shared__ uint64_t s_off[kNT];
    __shared__ uint32_t s_g[kNT];
    __shared__ int s_base[kNT];     // global id of the first group met
    __shared__ int s_tw[kNT];       // width of the met groups
    __shared__ int s_tx[kNT];       // groups per row of the view
    __shared__ uint2 s_rc[kNT];     // tile rectangle relative to the first group's first tile (x_lo | x_hi << 16, ...)
    __shared__ uint32_t s_first;
    const uint64_t stored = counters[2];          // min(instances, capacity)
    const uint64_t ob = (uint64_t)blockIdx.x * kEmitPerBlock;
    if (ob >= stored) return;
    const uint64_t oe = ob + kEmitPerBlock < stored ? ob + kEmitPerBlock : stored;
    const uint32_t n_vis = counters[0];
    const uint64_t total = *total64;
    if (threadIdx.x == 0) s_first = starts[blockIdx.x];
    __syncthreads();
    for (uint32_t e0 = s_first;; e0 += kNT) {
        const uint32_t i = e0 + threadIdx.x;
        if (i < n_vis) {
            const uint32_t rec = vis_vals[i];
            const int v = (int)(rec / (uint32_t)N);
            const ushort4 rc = rect_sorted[i];
            // tile sides 2^tsx x 2^tsy pixels
            const int tx0 = rc.x >> tsx, tx1 = rc.y >> tsx, ty0 = rc.z >> tsy, ty1 = rc.w >> tsy;
            const int gx0 = tx0 / GS, gx1 = tx1 / GS, gy0 = ty0 / GS;
            const sr_camera& c = cams[v];
            s_off[threadIdx.x] = offs[i];
            s_g[threadIdx.x] = rec - (uint32_t)v * (uint32_t)N;
            s_base[threadIdx.x] = c.group_offset + gy0 * c.groups_x + gx0;
            s_tw[threadIdx.x] = gx1 - gx0 + 1;
            s_tx[threadIdx.x] = c.groups_x;
            const int ox = GS * gx0, oy = GS * gy0;
            s_rc[threadIdx.x] = make_uint2((uint32_t)(tx0 - ox) | ((uint32_t)(tx1 - ox) << 16),
                                           (uint32_t)(ty0 - oy) | ((uint32_t)(ty1 - oy) << 16));
        } else {
            s_off[threadIdx.x] = ~0ull;
        }
        __syncthreads();
        const uint64_t wend = (e0 + kNT < n_vis) ? offs[e0 + kNT] : total;
        const uint64_t lo_o = ob > s_off[0] ? ob : s_off[0];
        const uint64_t hi_o = oe < wend ? oe : wend;
        for (uint64_t o = lo_o + threadIdx.x; o < hi_o; o += kNT) {
            int lo = 0, hi = kNT - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= o) lo = mid; else hi = mid - 1;
            }
            const uint32_t k = (uint32_t)(o - s_off[lo]);
            const uint32_t tw = (uint32_t)s_tw[lo];
            const uint32_t row = k / tw, colx = k - row * tw;
            inst_keys[o] = (uint32_t)s_base[lo] + row * (uint32_t)s_tx[lo] + colx;
            // the tile rectangle clipped to this group, in its tile coordinates
            const uint2 rr = s_rc[lo];
            const int x0 = (int)(rr.x & 0xffffu) - GS * (int)colx, x1 = (int)(rr.x >> 16) - GS * (int)colx;
            const int y0 = (int)(rr.y & 0xffffu) - GS * (int)row, y1 = (int)(rr.y >> 16) - GS * (int)row;
            const uint32_t sub = (uint32_t)(x0 > 0 ? x0 : 0) | ((uint32_t)(x1 < GS - 1 ? x1 : GS - 1) << 2) |
                                 ((uint32_t)(y0 > 0 ? y0 : 0) << 4) | ((uint32_t)(y1 < GS - 1 ? y1 : GS - 1) << 6);
            inst_vals[o] = s_g[lo] | (sub << SR_INST_ID_BITS);
        }
        if (wend >= oe || e0 + kNT >= n_vis) break;
        __syncthreads();
    }
}

// The sorted 64-bit keys (group id << 32 | depth key).
__global__ void __launch_bounds__(kNT)
k_keys64(const uint32_t* __restrict__ counters, const uint32_t* __restrict__ keys,
         const uint32_t* __restrict__ vals, uint64_t* __restrict__ keys64, const uint32_t* __restrict__ depth_key,
         const sr_camera* __restrict__ cams, int V, int N) {
    const uint32_t n = counters[2];
    for (uint32_t i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
        const uint32_t t = keys[i];
        const int v = view_of_group(cams, V, (int)t);
        keys64[i] = ((uint64_t)t << 32) | depth_key[(size_t)v * N + (vals[i] & kInstIdMask)];
    }
}

// Per tile, [start, end) of its group's run by binary search of the sorted
// group keys, one thread per tile; empty groups give [0, 0).
__global__ void __launch_bounds__(kNT)
k_ranges_search(const uint32_t* __restrict__ counters, const uint32_t* __restrict__ keys, int total_tiles,
                const sr_camera* __restrict__ cams, int V, uint2* __restrict__ ranges) {
    constexpr int GS = SR_TILE_GROUP;
    const int tile = (int)(blockIdx.x * kNT + threadIdx.x);
    if (tile >= total_tiles) return;
    const sr_camera& c = cams[view_of_tile(cams, V, tile)];
    const int local = tile - c.tile_offset;
    const int ty = local / c.tiles_x, tx = local - ty * c.tiles_x;
    const int t = c.group_offset + (ty / GS) * c.groups_x + tx / GS;
    const uint32_t n = counters[2];
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    const uint32_t s = lo;
    hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] <= (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    ranges[tile] = s < lo ? make_uint2(s, lo) : make_uint2(0u, 0u);
}

// dst[0, *count) = src[0, *count)
__global__ void k_copy_u32(const uint32_t* __restrict__ count, const uint32_t* __restrict__ src,
                           uint32_t* __restrict__ dst) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Blocks of a radix pass: one sub-tile each for small inputs, at most 4096
// (16 per CU) for large ones; the digit histogram is 256 x G counters.
constexpr int kMaxRadixBlocks = 4096;
int grid_for(uint64_t elems) {
    uint64_t g = (elems + kTile - 1) / kTile;
    if (g < 1) g = 1;
    if (g > kMaxRadixBlocks) g = kMaxRadixBlocks;
    return (int)g;
}

struct BinWs {
    uint32_t *vk0, *vv0, *vk1, *vv1;     // visible pairs, ping-pong
    uint32_t *ik0, *iv0, *ik1, *iv1;     // instances, ping-pong
    uint32_t *hist, *tot, *vsum, *tts, *estart;
    uint64_t *isum, *ioff, *itotal;
    ushort4* rsort;                      // rectangles of the visible pairs in depth order
    size_t bytes;
};

BinWs carve(void* base, uint64_t VN, uint64_t cap) {
    BinWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = (char*)base + off;
        off += align256(bytes);
        return (void*)p;
    };
    w.vk0 = (uint32_t*)take(VN * 4); w.vv0 = (uint32_t*)take(VN * 4);
    w.vk1 = (uint32_t*)take(VN * 4); w.vv1 = (uint32_t*)take(VN * 4);
    w.ik0 = (uint32_t*)take(cap * 4); w.iv0 = (uint32_t*)take(cap * 4);
    w.ik1 = (uint32_t*)take(cap * 4); w.iv1 = (uint32_t*)take(cap * 4);
    w.hist = (uint32_t*)take((uint64_t)kMaxRadix * kMaxRadixBlocks * 4);
    w.tot = (uint32_t*)take(kMaxRadix * 4);
    w.vsum = (uint32_t*)take(kMaxRadixBlocks * 4);
    w.isum = (uint64_t*)take(kMaxRadixBlocks * 8);
    w.ioff = (uint64_t*)take(VN * 8);
    w.tts = (uint32_t*)take(VN * 4);
    w.rsort = (ushort4*)take(VN * 8);
    w.estart = (uint32_t*)take(((cap + kEmitPerBlock - 1) / kEmitPerBlock) * 4);
    w.itotal = (uint64_t*)take(8);
    w.bytes = off;
    return w;
}

// Stable sort of `count` (device) pairs on bits [0, nbits), ping-ponging
// between (k0, v0) and (k1, v1); the last pass writes the values to
// vals_dst.  Returns the buffer holding the sorted keys.
uint32_t* radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* vals_dst,
                     const uint32_t* count, uint64_t cap, int nbits, uint32_t* hist, uint32_t* tot,
                     hipStream_t s) {
    const int G = grid_for(cap);
    const int passes = (nbits + kMaxDigitBits - 1) / kMaxDigitBits;
    if (passes == 0) {
        hipLaunchKernelGGL(k_copy_u32, dim3(1024), dim3(256), 0, s, count, v0, vals_dst);
        return k0;
    }
    // digits as even as possible, the narrower ones first (the first pass
    // reads the keys in emission order)
    const int per_lo = nbits / passes, wide_from = passes - nbits % passes;
    uint32_t *sk = k0, *sv = v0;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        const int bits = per_lo + (p >= wide_from ? 1 : 0);
        const bool last = p == passes - 1;
        uint32_t* dk = sk == k0 ? k1 : k0;
        uint32_t* dv = last ? vals_dst : (sv == v0 ? v1 : v0);
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kNT), 0, s, sk, count, G, shift, bits, hist);
        hipLaunchKernelGGL(k_radix_digit_scan, dim3(1 << bits), dim3(kNT), 0, s, hist, G, tot);
        // sub-tiles of 4096 (a sweep over 2048..8192 per pass: the fastest)
        hipLaunchKernelGGL(k_radix_scatter<16>, dim3(G), dim3(kNT), 0, s, sk, sv, count, G, shift, bits, hist, tot,
                           dk, dv);
        sk = dk;
        sv = dv;
        shift += bits;
    }
    return sk;
}

}  // namespace

size_t bin_workspace_bytes(uint64_t VN, uint64_t cap) { return carve(nullptr, VN, cap).bytes; }

hipError_t launch_bin_and_sort(const sr_config& cfg, int N, int V, int total_tiles, int total_groups,
                               const sr_camera* cams_dev,
                               const uint16_t* rect, const uint32_t* tiles_touched, const uint32_t* depth_key,
                               void* workspace, uint32_t cap, uint32_t* vals, uint64_t* keys64, uint32_t* ranges,
                               uint32_t* counters, uint32_t* status, bool count_only, hipStream_t s) {
    const uint64_t VN = (uint64_t)V * (uint64_t)N;
    // pixel sides of a tile group as powers of two (a group is 4 x 4 tiles)
    static_assert(SR_TILE_GROUP == 4, "group sides are two bits of tile coordinates");
    int gsx = 0, gsy = 0;
    while ((1 << gsx) < SR_TILE_GROUP * cfg.tile_w) ++gsx;
    while ((1 << gsy) < SR_TILE_GROUP * cfg.tile_h) ++gsy;
    if ((1 << gsx) != SR_TILE_GROUP * cfg.tile_w || (1 << gsy) != SR_TILE_GROUP * cfg.tile_h)
        return hipErrorInvalidValue;
    BinWs w = carve(workspace, VN, cap);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, counters, 0u, (uint64_t)SR_COUNTERS);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, ranges, 0u, 2ull * (uint64_t)total_tiles);
    if (VN == 0) return hipGetLastError();
    // 1. compact the visible pairs in (view, surfel) order
    const int Gv = grid_for(VN);
    hipLaunchKernelGGL(k_vis_count, dim3(Gv), dim3(kNT), 0, s, VN, Gv, tiles_touched, w.vsum);
    hipLaunchKernelGGL(k_scan_small<uint32_t>, dim3(1), dim3(kNT), 0, s, w.vsum, Gv, counters, 0, cap, w.itotal);
    hipLaunchKernelGGL(k_vis_compact, dim3(Gv), dim3(kNT), 0, s, VN, Gv, tiles_touched, depth_key, w.vsum,
                       w.vk0, w.vv0);
    // 2. stable sort by the 32 depth bits (ties keep (view, surfel) order):
    //    four 8-bit passes, the result ends in (vk0, vv0)
    {
        const int G = grid_for(VN);
        uint32_t *sk = w.vk0, *sv = w.vv0, *dk = w.vk1, *dv = w.vv1;
        for (int p = 0; p < 4; ++p) {
            hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kNT), 0, s, sk, counters, G, 8 * p, 8, w.hist);
            hipLaunchKernelGGL(k_radix_digit_scan, dim3(256), dim3(kNT), 0, s, w.hist, G, w.tot);
            // sub-tiles of 2048 pairs (8 per digit on average): faster than
            // 1024, 4096 or 8192 in a sweep on the 1M-surfel, 16-view batch
            // the sorted depth keys themselves are not used after the last pass
            hipLaunchKernelGGL(k_radix_scatter<8>, dim3(G), dim3(kNT), 0, s, sk, sv, counters, G, 8 * p, 8, w.hist,
                               w.tot, p == 3 ? nullptr : dk, dv);
            uint32_t* t;
            t = sk; sk = dk; dk = t;
            t = sv; sv = dv; dv = t;
        }
    }
    // after four passes the sorted pairs are in (vk0, vv0)
    // 3. instance offsets and emission in depth order
    const int Gi = Gv;
    hipLaunchKernelGGL(k_inst_count, dim3(Gi), dim3(kNT), 0, s, counters, Gi, w.vv0, (const ushort4*)rect, gsx, gsy,
                       w.tts, w.rsort, w.isum);
    hipLaunchKernelGGL(k_scan_small<uint64_t>, dim3(1), dim3(kNT), 0, s, w.isum, Gi, counters, 1, cap, w.itotal,
                       count_only ? nullptr : status);
    if (count_only) return hipGetLastError();     // the instance count is all that was asked for
    hipLaunchKernelGGL(k_inst_offsets, dim3(Gi), dim3(kNT), 0, s, counters, Gi, w.tts, w.isum, w.ioff);
    const uint64_t emit_blocks = ((uint64_t)cap + kEmitPerBlock - 1) / kEmitPerBlock;
    if (emit_blocks > 0) {
        hipLaunchKernelGGL(k_emit_starts, dim3((unsigned)((emit_blocks + kNT - 1) / kNT)), dim3(kNT), 0, s, counters,
                           w.ioff, (uint32_t)emit_blocks, w.estart);
        hipLaunchKernelGGL(k_emit, dim3((unsigned)emit_blocks), dim3(kNT), 0, s, counters, w.itotal, N,
                           gsx - 2, gsy - 2, cams_dev, w.vv0, (const ushort4*)w.rsort, w.ioff, w.estart, w.ik0, w.iv0);
    }
    // 4. stable sort by group id; values land in the caller's array
    int nbits = 0;
    while ((1ull << nbits) < (uint64_t)total_groups) ++nbits;
    uint32_t* sorted_keys = radix_sort(w.ik0, w.iv0, w.ik1, w.iv1, vals, counters + 2, cap, nbits, w.hist,
                                       w.tot, s);
    if (total_tiles > 0)
        hipLaunchKernelGGL(k_ranges_search, dim3((total_tiles + kNT - 1) / kNT), dim3(kNT), 0, s, counters,
                           sorted_keys, total_tiles, cams_dev, V, (uint2*)ranges);
    if (keys64) {
        const uint64_t rblocks = ((uint64_t)cap + kNT - 1) / kNT;
        hipLaunchKernelGGL(k_keys64, dim3((unsigned)(rblocks < 1 ? 1 : (rblocks > 65535 ? 65535 : rblocks))),
                           dim3(kNT), 0, s, counters, sorted_keys, vals, keys64, depth_key, cams_dev, V, N);
    }
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(n < 1024 * 256 ? (unsigned)((n + 255) / 256) : 1024u), dim3(256), 0, s, p, v,
                       n);
    return hipGetLastError();
}

namespace {

// Cameras [v0, v0 + Vc) of a batch laid out together, as a batch of their
// own: the tile, pixel and group offsets restart at zero.
__global__ void k_rebase_cams(const sr_camera* __restrict__ src, int Vc, sr_camera* __restrict__ dst) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Vc) return;
    sr_camera c = src[v];
    c.tile_offset -= src[0].tile_offset;
    c.pix_offset -= src[0].pix_offset;
    c.group_offset -= src[0].group_offset;
    dst[v] = c;
}

}  // namespace

hipError_t launch_rebase_cams(const sr_camera* src, int Vc, sr_camera* dst, hipStream_t s) {
    if (Vc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rebase_cams, dim3((Vc + 63) / 64), dim3(64), 0, s, src, Vc, dst);
    return hipGetLastError();
}

// ---- tile dispatch order ------------------------------------------------------
//
// Tiles sorted by descending cost class (ties keep ascending tile id), for a
// launch that takes its heaviest tiles first: the per-tile cost varies by
// two orders of magnitude, and a heavy tile dispatched late leaves the rest
// of the chip idle at the end of the grid.  The order only has to be
// approximately longest-first, so the cost is reduced to a 9-bit
// logarithmic class (costs below 16 exact, above that 16 classes per
// octave: within about 6 %) and sorted in one radix pass.

namespace {

constexpr int kOrderBits = 9;

__device__ __forceinline__ uint32_t cost_class(uint32_t c) {
    if (c < 16u) return c;
    const uint32_t e = 31u - (uint32_t)__builtin_clz(c);       // msb position, >= 4
    return (e - 3u) * 16u + ((c >> (e - 4u)) & 15u);           // <= 28 * 16 + 15 = 463
}

__global__ void k_order_keys(int T, const uint32_t* __restrict__ cost, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ ids, uint32_t* __restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *count = (uint32_t)T;
    if (i < T) {
        keys[i] = ((1u << kOrderBits) - 1u) - cost_class(cost[i]);    // ascending key = descending cost
        ids[i] = (uint32_t)i;
    }
}

struct OrderWs {
    uint32_t *k0, *v0, *k1, *v1, *hist, *tot, *count;
};

size_t order_ws_layout(int T, void* base, OrderWs* w) {
    const uint64_t G = (uint64_t)grid_for((uint64_t)T);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> uint32_t* {
        uint32_t* p = base ? (uint32_t*)((char*)base + off) : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    w->k0 = take((uint64_t)T * 4);
    w->v0 = take((uint64_t)T * 4);
    w->k1 = take((uint64_t)T * 4);
    w->v1 = take((uint64_t)T * 4);
    w->hist = take((uint64_t)kMaxRadix * G * 4);
    w->tot = take(kMaxRadix * 4);
    w->count = take(4);
    return (size_t)off;
}

}  // namespace

size_t tile_order_workspace(int T) {
    OrderWs w;
    return order_ws_layout(T, nullptr, &w);
}

hipError_t launch_tile_order(int T, const uint32_t* cost, void* ws, uint32_t* order, hipStream_t s) {
    if (T == 0) return hipSuccess;
    OrderWs w;
    order_ws_layout(T, ws, &w);
    hipLaunchKernelGGL(k_order_keys, dim3((T + kNT - 1) / kNT), dim3(kNT), 0, s, T, cost, w.k0, w.v0, w.count);
    radix_sort(w.k0, w.v0, w.k1, w.v1, order, w.count, (uint64_t)T, kOrderBits, w.hist, w.tot, s);
    return hipGetLastError();
}

}  // namespace sr
