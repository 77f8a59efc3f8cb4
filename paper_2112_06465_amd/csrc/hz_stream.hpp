// Bandwidth calibration kernels: a read-only stream and a copy over a flat
// buffer, each thread keeping kStreamU independent 16-byte loads in flight.
// They measure the memory ceiling that the library's bandwidth-bound kernels
// are compared against on the same part (the paper repeats every operation
// and averages, Section 3.3; a ceiling measured the same way makes the
// fraction of peak meaningful on this hardware).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hz {

constexpr int kStreamBlock = 256;   // threads per block (4 waves)
constexpr int kStreamU = 8;         // 16-byte loads in flight per thread
constexpr int kStreamGrid = 2048;   // blocks (8 per CU); also the partial count of the read

// Sum of the doubles of p[0, n16) (16-byte elements) into part[blockIdx.x].
// Whole chunks of kStreamBlock * kStreamU elements are read with straight-line
// loads (chunk c by block c mod G); the ragged tail by the last block, guarded.
__global__ __launch_bounds__(kStreamBlock) void k_stream_read(const double2* __restrict__ p, int64_t n16,
                                                              double* __restrict__ part) {
    constexpr int64_t C = int64_t(kStreamBlock) * kStreamU;
    const int64_t full = n16 / C;
    double acc = 0.0;
    for (int64_t c = blockIdx.x; c < full; c += gridDim.x) {
        const double2* q = p + c * C + threadIdx.x;
        double2 v[kStreamU];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) v[u] = q[u * kStreamBlock];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) acc += v[u].x + v[u].y;
    }
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = full * C + threadIdx.x; i < n16; i += kStreamBlock) acc += p[i].x + p[i].y;
    // fixed-order block sum: wave tree, then the 4 wave totals in order
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

// *out = sum of part[0, G) in index order (one block).
__global__ __launch_bounds__(kStreamBlock) void k_stream_fin(const double* __restrict__ part, int G,
                                                             double* __restrict__ out) {
    __shared__ double w[kStreamBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < G; i += kStreamBlock) acc += part[i];
    w[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < kStreamBlock; ++k) s += w[k];
        *out = s;
    }
}

// dst[0, n16) = src[0, n16), 16-byte elements, same chunking as the read.
__global__ __launch_bounds__(kStreamBlock) void k_stream_copy(const double2* __restrict__ src, int64_t n16,
                                                              double2* __restrict__ dst) {
    constexpr int64_t C = int64_t(kStreamBlock) * kStreamU;
    const int64_t full = n16 / C;
    for (int64_t c = blockIdx.x; c < full; c += gridDim.x) {
        const int64_t i0 = c * C + threadIdx.x;
        double2 v[kStreamU];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) v[u] = src[i0 + u * kStreamBlock];
#pragma unroll
        for (int u = 0; u < kStreamU; ++u) dst[i0 + u * kStreamBlock] = v[u];
    }
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = full * C + threadIdx.x; i < n16; i += kStreamBlock) dst[i] = src[i];
}

}  // namespace hz
