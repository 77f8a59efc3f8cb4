// Standalone BLAS-1 kernels (zaxpy, zdotc, dznrm2 of the C-ABI), the paper's
// basic operations (Section 5: axpy, dot product, 2-norm).
//
// Each is one streaming pass: the vectors are cut into chunks of kB1Block *
// kB1U complex elements (16 KiB per vector), one chunk per block, each thread
// issuing its kB1U loads of a chunk straight-line and non-temporal (every
// instruction reads 256 consecutive elements, whole cache lines) before using
// any of them.  A ragged tail is handled by the last block with guarded
// accesses.
//
// A reduction finishes in the same launch without a memory fence.  Each block
// sums its elements in a fixed order (per thread in element order, a wave
// tree, then the block's waves in order) and publishes the total with one
// agent-scope atomic store into a slot of its own, a 64-bit word that holds a
// signalling-NaN marker while empty.  The last block of the grid reads every
// slot with agent-scope atomic loads until none holds the marker, adds the
// totals in index order, writes the result and puts the marker back.  Only the
// coherence of each single word is relied on (a load of a word that was stored
// once returns the stored value or an older one, never a mix), so no release
// or acquire ordering between different words is needed.  (The alternative, a
// ticket counter with a device-scope release fence in every block, writes back
// the XCD's L2 on this multi-XCD part: that dot product measured 1.6 to 2.4
// times slower than two launches, and two launches 1.3 times slower than the
// slots in a captured graph.)  A computed total that is a NaN is stored as the
// quiet NaN, so no total can equal the marker.  No floating-point atomics:
// results are bitwise reproducible and equal to a sum of the same partials
// by a separate finishing kernel.
//
// The last block's wait ends when all blocks have stored, which needs only
// that they are scheduled; as a guard it also ends after `limit` ticks of the
// constant-rate wall clock.  A wait that ends that way writes a NaN result and
// sets the handle's broken word: every later reduction on the handle then
// writes NaN without waiting (a late store could otherwise leave a stale total
// in a slot), until the slots are armed again.  A limit of 0 takes that path
// at once, so that it can be exercised without a stalled block.
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
// Whole chunks are software-pipelined: chunk j + 1's loads are issued before
// chunk j's stores.  One in-order counter tracks loads and stores on this
// architecture, so with the stores first the wait for the next chunk's loads
// would also wait for them.
__global__ __launch_bounds__(kB1Block) void k_zaxpy_s(int64_t n, int per, double2 alpha, const double2* x,
                                                      double2* y) {
    const int64_t c0 = int64_t(blockIdx.x) * per;  // the block's first chunk
    int64_t chunks = (n / kB1Chunk) - c0;           // whole chunks of this block
    if (chunks > per) chunks = per;
    if (chunks < 0) chunks = 0;
    double2 xv[kB1U], yv[kB1U];
    auto load = [&](int64_t c) {
        const int64_t i0 = c * kB1Chunk + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kB1U; ++u) xv[u] = ld_nt(x + i0 + u * kB1Block);
#pragma unroll
        for (int u = 0; u < kB1U; ++u) yv[u] = ld_nt(y + i0 + u * kB1Block);
    };
    if (chunks > 0) load(c0);
    for (int64_t j = 0; j < chunks; ++j) {
        const int64_t i0 = (c0 + j) * kB1Chunk + threadIdx.x;
        double2 r[kB1U];
#pragma unroll
        for (int u = 0; u < kB1U; ++u) r[u] = cfma<double>(alpha, xv[u], yv[u]);
        if (j + 1 < chunks) load(c0 + j + 1);
#pragma unroll
        for (int u = 0; u < kB1U; ++u) st_nt(y + i0 + u * kB1Block, r[u]);
    }
    // the ragged tail past the last whole chunk, in the block that owns that chunk
    const int64_t full = n / kB1Chunk;
    if (full >= c0 && full < c0 + per) {
        for (int64_t i = full * kB1Chunk + threadIdx.x; i < n; i += kB1Block) y[i] = cfma<double>(alpha, x[i], y[i]);
    }
}

constexpr unsigned long long kB1SlotEmpty = 0x7ff4dead0000beefull;  // a signalling NaN no arithmetic yields

__device__ __forceinline__ unsigned long long b1_slot_bits(double v) {
    if (v != v) v = __builtin_nan("");
    return static_cast<unsigned long long>(__double_as_longlong(v));
}

// Slots (2 kB1MaxGrid words) and the broken word of a handle.
struct B1Slots {
    unsigned long long* slot;
    unsigned* broken;
    unsigned long long limit;  // wall-clock ticks the last block waits at most; 0: give up at once
};

// Marks every slot empty and clears the broken word.
__global__ __launch_bounds__(kB1Block) void k_b1_arm(B1Slots s) {
    const int i = blockIdx.x * kB1Block + threadIdx.x;
    if (i < 2 * kB1MaxGrid) s.slot[i] = kB1SlotEmpty;
    if (i == 0) *s.broken = 0u;
}

// MODE 0: *out = sum conj(x_i) y_i (complex, K = 2 components); MODE 1:
// *out = sqrt(sum |x_i|^2) (K = 1).  Block b's total of component k goes to
// slot k G + b.
template <int MODE>
__global__ __launch_bounds__(kB1Block) void k_zdot_s(int64_t n, int per, const double2* __restrict__ x,
                                                     const double2* __restrict__ y, B1Slots sl, void* out) {
    constexpr int K = MODE == 0 ? 2 : 1;
    const int G = gridDim.x;
    // a previous wait that timed out: no slot is trusted any more (read early, used at the end)
    const unsigned broken = threadIdx.x == 0 ? __hip_atomic_load(sl.broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                             : 0u;
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
    __shared__ unsigned skip;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = e[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) w[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        skip = broken;
        if (!broken) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double s = (w[k][0] + w[k][1]) + (w[k][2] + w[k][3]);
                __hip_atomic_store(sl.slot + int64_t(k) * G + blockIdx.x, b1_slot_bits(s), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (blockIdx.x != G - 1) return;
    __syncthreads();  // `skip` and the reuse of w below
    bool late = skip != 0u || sl.limit == 0;
    const uint64_t t0 = wall_clock64();
    // slot i of every component is loaded at once (one round trip to L2 for all K), then each is
    // waited for in turn; per component the slots are added in index order
    double tot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = 0.0;
    for (int i = threadIdx.x; i < G && !late; i += kB1Block) {
        unsigned long long u[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            u[k] = __hip_atomic_load(sl.slot + int64_t(k) * G + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            while (!late && u[k] == kB1SlotEmpty) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > sl.limit) {
                    late = true;
                    break;
                }
                u[k] = __hip_atomic_load(sl.slot + int64_t(k) * G + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (late) break;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            tot[k] += __longlong_as_double(static_cast<long long>(u[k]));
            __hip_atomic_store(sl.slot + int64_t(k) * G + i, kB1SlotEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) tot[k] += __shfl_down(tot[k], off, 64);
    const bool any_late = __syncthreads_or(late);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if ((threadIdx.x & 63) == 0) w[k][threadIdx.x >> 6] = tot[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            s[k] = any_late ? __builtin_nan("") : (w[k][0] + w[k][1]) + (w[k][2] + w[k][3]);
        if constexpr (MODE == 0) {
            static_cast<double2*>(out)[0] = mk<double>(s[0], s[1]);
        } else {
            static_cast<double*>(out)[0] = __builtin_sqrt(s[0]);
        }
        if (any_late) __hip_atomic_store(sl.broken, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace hz
