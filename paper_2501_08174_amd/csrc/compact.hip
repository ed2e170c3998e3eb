// Stream compaction of the per-surfel arrays: the pruning decided by the
// occlusion statistics (Section 4.3), optionally with a minimum opacity,
// applied to the parameters (and whatever else the caller keeps per surfel,
// such as optimiser moments).  Stable: kept surfels keep their order.
//
// Pass 1 counts the kept surfels of every chunk; a single block scans the
// chunk counts; pass 2 re-derives each surfel's rank inside its chunk with a
// block scan and copies its rows of every array.
#include "common.h"
#include "launch.h"

namespace sr {

namespace {

constexpr int kNT = 256;
constexpr int kChunk = 8192;          // surfels per block
constexpr int kMaxArrays = SR_COMPACT_MAX_ARRAYS;

struct CompactArrays {
    const float* src[kMaxArrays];
    float* dst[kMaxArrays];
    int width[kMaxArrays];
    int n;
};

__device__ __forceinline__ bool kept(int64_t i, const uint8_t* __restrict__ prune, const float* __restrict__ opac,
                                     float min_opac) {
    return !prune[i] && (opac == nullptr || opac[i] >= min_opac);
}

__global__ void __launch_bounds__(kNT)
k_compact_count(int N, const uint8_t* __restrict__ prune, const float* __restrict__ opac, float min_opac,
                uint32_t* __restrict__ counts) {
    __shared__ uint32_t s[kNT];
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    const int64_t e = b + kChunk < N ? b + kChunk : N;
    uint32_t c = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += kNT) c += kept(i, prune, opac, min_opac) ? 1u : 0u;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = kNT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// exclusive scan of the chunk counts in place (one block); total to *n_kept
__global__ void __launch_bounds__(kNT)
k_compact_scan(int nchunk, uint32_t* __restrict__ counts, uint32_t* __restrict__ n_kept) {
    __shared__ uint32_t s[kNT];
    uint32_t carry = 0;
    for (int base = 0; base < nchunk; base += kNT) {
        const int i = base + (int)threadIdx.x;
        const uint32_t v = i < nchunk ? counts[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kNT; off <<= 1) {         // inclusive Hillis-Steele scan
            const uint32_t t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunk) counts[i] = carry + s[threadIdx.x] - v;
        carry += s[kNT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_kept = carry;
}

__global__ void __launch_bounds__(kNT)
k_compact_copy(int N, const uint8_t* __restrict__ prune, const float* __restrict__ opac, float min_opac,
               const uint32_t* __restrict__ offs, CompactArrays arr) {
    __shared__ uint32_t s[kNT];
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    const int64_t e = b + kChunk < N ? b + kChunk : N;
    uint32_t run = offs[blockIdx.x];
    for (int64_t base = b; base < e; base += kNT) {
        const int64_t i = base + threadIdx.x;
        const bool k = i < e && kept(i, prune, opac, min_opac);
        s[threadIdx.x] = k ? 1u : 0u;
        __syncthreads();
        for (int off = 1; off < kNT; off <<= 1) {
            const uint32_t t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (k) {
            const uint32_t j = run + s[threadIdx.x] - 1u;
            for (int a = 0; a < arr.n; ++a) {
                const int w = arr.width[a];
                const float* src = arr.src[a] + (size_t)i * w;
                float* dst = arr.dst[a] + (size_t)j * w;
                for (int c = 0; c < w; ++c) dst[c] = src[c];
            }
        }
        run += s[kNT - 1];
        __syncthreads();
    }
}

}  // namespace

size_t compact_workspace_bytes(int N) { return (size_t)((N + kChunk - 1) / kChunk + 1) * sizeof(uint32_t); }

hipError_t launch_compact(int N, const uint8_t* prune, const float* opac, float min_opac, int n_arrays,
                          const float* const* src, float* const* dst, const int* widths, void* ws,
                          uint32_t* n_kept, hipStream_t s) {
    CompactArrays arr{};
    arr.n = n_arrays;
    for (int a = 0; a < n_arrays; ++a) {
        arr.src[a] = src[a];
        arr.dst[a] = dst[a];
        arr.width[a] = widths[a];
    }
    const int nchunk = (N + kChunk - 1) / kChunk;
    uint32_t* counts = (uint32_t*)ws;
    if (N == 0) {
        hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kNT), 0, s, 0, counts, n_kept);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_compact_count, dim3(nchunk), dim3(kNT), 0, s, N, prune, opac, min_opac, counts);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kNT), 0, s, nchunk, counts, n_kept);
    hipLaunchKernelGGL(k_compact_copy, dim3(nchunk), dim3(kNT), 0, s, N, prune, opac, min_opac,
                       (const uint32_t*)counts, arr);
    return hipGetLastError();
}

}  // namespace sr
