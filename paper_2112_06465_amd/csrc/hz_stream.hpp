// Bandwidth calibration kernels: a read-only stream and a copy over a flat
// buffer.  They measure the memory ceiling that the library's bandwidth-bound
// kernels are compared against on the same part (the paper repeats every
// operation and averages, Section 3.3; a ceiling measured the same way makes
// the fraction of peak meaningful on this hardware).
//
// The buffer is cut into chunks of kStreamBlock * kStreamU 16-byte elements
// (32 KiB); block b takes `per` consecutive chunks, each thread issuing its
// kStreamU loads of a chunk straight-line and non-temporal (the data is read
// once: streaming loads keep it from displacing cached data, and on this part
// they sustain about 10 % more bandwidth than ordinary loads).  The ragged
// tail past the last whole chunk is read by the last block, guarded.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hz {

constexpr int kStreamBlock = 256;       // threads per block (4 waves)
static_assert(kStreamBlock == 256, "the finishing kernels add four wave totals");
constexpr int kStreamU = 8;             // 16-byte loads in flight per thread
constexpr int kStreamMaxGrid = 5120;    // at most this many blocks (= partials of the read)

typedef double stream_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ stream_d2 stream_ld(const double2* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const stream_d2*>(p));
}

// Sum of the doubles of p[0, n16) into part[blockIdx.x]; the sum of a block
// is taken in a fixed order (per thread in chunk order, a wave tree, then the
// waves in order), so the total is bitwise reproducible.
__global__ __launch_bounds__(kStreamBlock) void k_stream_read(const double2* __restrict__ p, int64_t n16, int per,
                                                              double* __restrict__ part) {
    constexpr int64_t C = int64_t(kStreamBlock) * kStreamU;
    const int64_t full = n16 / C;
    double acc = 0.0;
    for (int j = 0; j < per; ++j) {
        const int64_t c = int64_t(blockIdx.x) * per + j;
        if (c >= full) break;
        const double2* q = p + c * C + threadIdx.x;
        stream_d2 v[kStreamU];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) v[u] = stream_ld(q + u * kStreamBlock);
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) acc += v[u].x + v[u].y;
    }
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = full * C + threadIdx.x; i < n16; i += kStreamBlock) acc += p[i].x + p[i].y;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double w[kStreamBlock / 64];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < kStreamBlock / 64; ++k) s += w[k];
        part[blockIdx.x] = s;
    }
}

// *out = sum of part[0, G) in a fixed order (one block): per thread over
// i, i + kStreamBlock, ..., a wave tree, then the four wave totals.
__global__ __launch_bounds__(kStreamBlock) void k_stream_fin(const double* __restrict__ part, int G,
                                                             double* __restrict__ out) {
    __shared__ double w[kStreamBlock / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < G; i += kStreamBlock) acc += part[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = (w[0] + w[1]) + (w[2] + w[3]);
}

// dst[0, n16) = src[0, n16), 16-byte elements, same chunking as the read.
__global__ __launch_bounds__(kStreamBlock) void k_stream_copy(const double2* __restrict__ src, int64_t n16, int per,
                                                              double2* __restrict__ dst) {
    constexpr int64_t C = int64_t(kStreamBlock) * kStreamU;
    const int64_t full = n16 / C;
    for (int j = 0; j < per; ++j) {
        const int64_t c = int64_t(blockIdx.x) * per + j;
        if (c >= full) break;
        const int64_t i0 = c * C + threadIdx.x;
        stream_d2 v[kStreamU];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) v[u] = stream_ld(src + i0 + u * kStreamBlock);
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) dst[i0 + u * kStreamBlock] = make_double2(v[u].x, v[u].y);
    }
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = full * C + threadIdx.x; i < n16; i += kStreamBlock) dst[i] = src[i];
}

// Launch shape for n16 elements: chunks per block and blocks (>= 1, <= kStreamMaxGrid).
struct StreamShape {
    int per, G;
};
inline StreamShape stream_shape(int64_t n16) {
    const int64_t chunks = n16 / (int64_t(kStreamBlock) * kStreamU);
    StreamShape s;
    s.per = int((chunks + kStreamMaxGrid - 1) / kStreamMaxGrid);
    if (s.per < 1) s.per = 1;
    const int64_t G = (chunks + s.per - 1) / s.per;
    s.G = G < 1 ? 1 : int(G);
    return s;
}

}  // namespace hz
