// Standalone BLAS-1 kernels (zaxpy, zdotc, dznrm2 of the C-ABI), the paper's
// basic operations (Section 5: axpy, dot product, 2-norm).
//
// Each is one streaming pass: the vectors are cut into chunks of kB1Block *
// kB1U complex elements (16 KiB per vector), one chunk per block, each thread
// issuing its kB1U loads of a chunk straight-line and non-temporal (every
// instruction reads 256 consecutive elements, whole cache lines) before using
// any of them.  A ragged tail is handled by the last block with guarded
// accesses.  A reduction writes one partial per block (per thread in element
// order, a wave tree, then the block's waves in order) and a one-block kernel
// adds the partials in index order.  (Finishing in the same launch, the last
// block to take an integer ticket adding the partials, needs a device-scope
// release fence in every block; on this multi-XCD part each such fence writes
// back and invalidates the XCD's L2, and the one-launch dot product measured
// 10x slower than two launches.)  No floating-point atomics: results are
// bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hz_kernels.hpp"

namespace hz {

constexpr int kB1Block = 256;  // threads per block
static_assert(kB1Block == 256, "the finishing kernels add four wave totals");
constexpr int kB1U = 4;        // elements per thread per chunk
constexpr int64_t kB1Chunk = int64_t(kB1Block) * kB1U;

constexpr int kB1MaxGrid = 2560;  // blocks at most of a reduction (partials per component)

// Launch shape for n elements: chunks per block and blocks.
struct B1Shape {
    int per, G;
};
inline B1Shape b1_shape(int64_t n) {
    const int64_t chunks = (n + kB1Chunk - 1) / kB1Chunk;
    B1Shape s;
    s.per = int((chunks + kB1MaxGrid - 1) / kB1MaxGrid);
    if (s.per < 1) s.per = 1;
    const int64_t G = (chunks + s.per - 1) / s.per;
    s.G = G < 1 ? 1 : int(G);
    return s;
}

__device__ __forceinline__ double2 ld_nt(const double2* p) { return ld_mat(p); }
__device__ __forceinline__ void st_nt(double2* p, double2 v) {
#if HZ_STREAM_MATRIX
    hz_d2v t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<hz_d2v*>(p));
#else
    *p = v;
#endif
}

// y = alpha x + y
// (x may equal y: every element is read before it is written, by the same thread)
__global__ __launch_bounds__(kB1Block) void k_zaxpy_s(int64_t n, int per, double2 alpha, const double2* x,
                                                      double2* y) {
  for (int j = 0; j < per; ++j) {
    const int64_t i0 = (int64_t(blockIdx.x) * per + j) * kB1Chunk + threadIdx.x;
    if (i0 >= n) break;
    if (i0 + (kB1U - 1) * kB1Block < n) {
        double2 xv[kB1U], yv[kB1U];
#pragma unroll
        for (int u = 0; u < kB1U; ++u) xv[u] = ld_nt(x + i0 + u * kB1Block);
#pragma unroll
        for (int u = 0; u < kB1U; ++u) yv[u] = ld_nt(y + i0 + u * kB1Block);
#pragma unroll
        for (int u = 0; u < kB1U; ++u) st_nt(y + i0 + u * kB1Block, cfma<double>(alpha, xv[u], yv[u]));
    } else {
        for (int u = 0; u < kB1U; ++u) {
            const int64_t i = i0 + u * kB1Block;
            if (i < n) y[i] = cfma<double>(alpha, x[i], y[i]);
        }
    }
  }
}

// Block partials of K components: part[k G + b].  MODE 0: conj(x_i) y_i
// (K = 2); MODE 1: |x_i|^2 (K = 1).
template <int MODE>
__global__ __launch_bounds__(kB1Block) void k_zdot_s(int64_t n, int per, const double2* __restrict__ x,
                                                     const double2* __restrict__ y, double* __restrict__ part) {
    constexpr int K = MODE == 0 ? 2 : 1;
    const int G = gridDim.x;
    double e[K];
#pragma unroll
    for (int k = 0; k < K; ++k) e[k] = 0.0;
    auto acc = [&](double2 xv, double2 yv) {
        if constexpr (MODE == 0) {
            const double2 c = cdotacc(xv.x, xv.y, yv.x, yv.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        } else {
            e[0] = __builtin_fma(xv.x, xv.x, e[0]);
            e[0] = __builtin_fma(xv.y, xv.y, e[0]);
        }
    };
    for (int j = 0; j < per; ++j) {
        const int64_t i0 = (int64_t(blockIdx.x) * per + j) * kB1Chunk + threadIdx.x;
        if (i0 >= n) break;
        if (i0 + (kB1U - 1) * kB1Block < n) {
            double2 xv[kB1U], yv[kB1U];
#pragma unroll
            for (int u = 0; u < kB1U; ++u) xv[u] = ld_nt(x + i0 + u * kB1Block);
            if constexpr (MODE == 0) {
#pragma unroll
                for (int u = 0; u < kB1U; ++u) yv[u] = ld_nt(y + i0 + u * kB1Block);
            }
#pragma unroll
            for (int u = 0; u < kB1U; ++u) acc(xv[u], MODE == 0 ? yv[u] : xv[u]);
        } else {
            for (int u = 0; u < kB1U; ++u) {
                const int64_t i = i0 + u * kB1Block;
                if (i < n) acc(x[i], MODE == 0 ? y[i] : x[i]);
            }
        }
    }
    __shared__ double w[K][kB1Block / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = e[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) w[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < kB1Block / 64; ++q) s += w[k][q];
            part[int64_t(k) * G + blockIdx.x] = s;
        }
    }
}

// The total of G partials per component (one block), in a fixed order: each
// thread sums partials i, i + kB1Block, ..., a wave tree combines the
// threads, thread 0 adds the four wave totals.  MODE 0 writes the complex
// sum, MODE 1 the square root of the sum.
template <int MODE>
__global__ __launch_bounds__(kB1Block) void k_zdot_fin(const double* __restrict__ part, int G, void* out) {
    constexpr int K = MODE == 0 ? 2 : 1;
    __shared__ double w[K][kB1Block / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int i = threadIdx.x; i < G; i += kB1Block) t += part[int64_t(k) * G + i];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if ((threadIdx.x & 63) == 0) w[k][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[K];
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] = (w[k][0] + w[k][1]) + (w[k][2] + w[k][3]);
        if constexpr (MODE == 0) {
            static_cast<double2*>(out)[0] = mk<double>(s[0], s[1]);
        } else {
            static_cast<double*>(out)[0] = __builtin_sqrt(s[0]);
        }
    }
}

}  // namespace hz
