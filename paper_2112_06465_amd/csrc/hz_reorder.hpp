// Level-set (breadth-first) reordering of a CSR matrix on the device.
//
// The solver's kernels gather x by column index.  When the caller's numbering
// scatters the neighbours of a row across the whole vector (a randomly
// numbered mesh), each gathered 16-byte element pulls a cache line from far
// away and the product becomes gather-bound.  Renumbering the unknowns by
// breadth-first level from a pseudo-peripheral node (a Cuthill-McKee-type
// ordering without the degree sort) puts the neighbours of every row within
// two adjacent level sets, so the x window of a block stays in its XCD's L2.
// BiCGStab with Jacobi scaling is invariant under a symmetric permutation
// P A P^T (all inner products are sums over the same index set), so the
// solve in the new numbering is the same method up to rounding order.
//
// Everything here is integer and index work and is bitwise reproducible:
//   * BFS levels are distances, independent of the order threads run in: a
//     level-L pass writes only the value L + 1, so racing writers agree;
//   * the order within a level is by the caller's index (a stable radix sort
//     of (level, index) on the host side), so the permutation is a pure
//     function of the pattern.
#pragma once

#include "hz_kernels.hpp"

namespace hz {

// level[i] = -1 except level[*start] = 0; active[0] = 1, active[1..n] = 0;
// *maxlev = 0.  Grid covers n + 1 items.
__global__ __launch_bounds__(kBlock) void k_bfs_seed(int n, const int* __restrict__ start, int* __restrict__ level,
                                                     int* __restrict__ active, int* __restrict__ maxlev) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int s0 = *start;
    if (i < n) level[i] = i == s0 ? 0 : -1;
    if (i <= n) active[i] = i == 0 ? 1 : 0;
    if (i == 0) *maxlev = 0;
}

// One breadth-first step: every node at level L labels its unlabelled
// neighbours L + 1.  active[L] says level L is not empty (written by the
// previous step, so it is read-only here); the step sets active[L + 1] and
// *maxlev = L + 1 when it labels anything.  Steps past the last level return
// at entry, so the host may enqueue more steps than there are levels.
__global__ __launch_bounds__(kBlock) void k_bfs_level(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                      int* level, int* __restrict__ active, int* __restrict__ maxlev,
                                                      int L) {
    if (L >= n || active[L] == 0) return;  // uniform over the grid
    int grew = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        if (level[i] != L) continue;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (level[j] < 0) {
                level[j] = L + 1;
                grew = 1;
            }
        }
    }
    if (__syncthreads_or(grew) && threadIdx.x == 0) {
        active[L + 1] = 1;
        *maxlev = L + 1;
    }
}

// *out = the smallest index at level Lmax (out starts at n).
__global__ __launch_bounds__(kBlock) void k_bfs_far(int n, const int* __restrict__ level, int Lmax,
                                                    int* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && level[i] == Lmax) atomicMin(out, (int)i);
}

// Sort keys: the level, with unreached nodes (other connected components)
// in a last bucket Lmax + 1; values: the caller's index.
__global__ __launch_bounds__(kBlock) void k_order_keys(int n, const int* __restrict__ level, int Lmax,
                                                       unsigned* __restrict__ key, int* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int l = level[i];
    key[i] = unsigned(l < 0 ? Lmax + 1 : l);
    idx[i] = (int)i;
}

// inv[perm[k]] = k
__global__ __launch_bounds__(kBlock) void k_invert(int n, const int* __restrict__ perm, int* __restrict__ inv) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) inv[perm[k]] = (int)k;
}

// len[0] = 0, len[k + 1] = length of the caller's row perm[k]
__global__ __launch_bounds__(kBlock) void k_perm_rowlen(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ perm, int* __restrict__ len) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k == 0) len[0] = 0;
    if (k < n) {
        const int o = perm[k];
        len[k + 1] = rp[o + 1] - rp[o];
    }
}

// Row k of P A P^T is the caller's row perm[k] with columns renumbered by
// inv; 8 lanes per row copy it (the columns are sorted afterwards).
__global__ __launch_bounds__(kBlock) void k_perm_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const double2* __restrict__ v, const int* __restrict__ perm,
                                                      const int* __restrict__ inv, const int* __restrict__ rp2,
                                                      int* __restrict__ ci2, double2* __restrict__ v2) {
    constexpr int L = 8;
    const int64_t k = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
    const int lane = threadIdx.x % L;
    if (k >= n) return;
    const int o = perm[k];
    const int b0 = rp[o], len = rp[o + 1] - b0, d0 = rp2[k];
    for (int e = lane; e < len; e += L) {
        ci2[d0 + e] = inv[ci[b0 + e]];
        v2[d0 + e] = v[b0 + e];
    }
}

// *bad = 1 unless 0 <= perm[k] < n and inv[perm[k]] = k for every k (then
// perm is a bijection and inv its inverse).
__global__ __launch_bounds__(kBlock) void k_check_perm(int n, const int* __restrict__ perm,
                                                       const int* __restrict__ inv, int* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int p = perm[k];
    if (p < 0 || p >= n || inv[p] != (int)k) *bad = 1;
}

// dst[k] = src[perm[k]]  (into the new numbering)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_perm(int n, const int* __restrict__ perm,
                                                        const cx<T>* __restrict__ src, cx<T>* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) dst[k] = src[perm[k]];
}

// dst[perm[k]] = src[k]  (back to the caller's numbering)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_perm(int n, const int* __restrict__ perm,
                                                         const cx<T>* __restrict__ src, cx<T>* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) dst[perm[k]] = src[k];
}

}  // namespace hz
