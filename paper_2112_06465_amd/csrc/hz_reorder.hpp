// Level-set (Cuthill-McKee) reordering of a CSR matrix on the device.
//
// The solver's kernels gather x by column index.  When the caller's numbering
// scatters the neighbours of a row across the whole vector (a randomly
// numbered mesh), each gathered 16-byte element pulls a cache line from far
// away and the product becomes gather-bound.  Renumbering the unknowns by
// breadth-first level from a pseudo-peripheral node puts the neighbours of
// every row within two adjacent level sets; ordering each level the
// Cuthill-McKee way (by the new position of the earliest neighbour on the
// previous level, then by degree) also keeps the neighbours of consecutive
// rows close together inside those levels, so a row's gathers share cache
// lines.  BiCGStab with Jacobi scaling is invariant under a symmetric
// permutation P A P^T (all inner products are sums over the same index set),
// so the solve in the new numbering is the same method up to rounding order.
//
// Everything here is integer and index work and is bitwise reproducible:
//   * BFS levels are distances, independent of the order threads run in: a
//     level-L pass writes only the value L + 1, so racing writers agree;
//   * levels are formed by a stable radix sort of (level, index); each level
//     is then sorted stably by (earliest new position of a neighbour on the
//     previous level, degree), level after level, so ties fall back to the
//     caller's index and the permutation is a pure function of the pattern.
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

// off[key] = first position of each key in the sorted keys skey[0..n); the
// last position also writes off[skey[n-1] + 1] = n.
__global__ __launch_bounds__(kBlock) void k_level_starts(int n, const unsigned* __restrict__ skey,
                                                         int* __restrict__ off) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const unsigned c = skey[k];
    if (k == 0 || skey[k - 1] != c) off[c] = (int)k;
    if (k == n - 1) off[c + 1] = n;
}

// Cuthill-McKee keys of the m nodes of level L (given in index order): the
// smallest new position pos[u] of a neighbour u on level L - 1 (n when there
// is none), shifted left by 8, plus the degree capped at 255.
__global__ __launch_bounds__(kBlock) void k_cm_keys(int m, const int* __restrict__ nodes, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const int* __restrict__ level, int L,
                                                    const int* __restrict__ pos, int n,
                                                    unsigned long long* __restrict__ key, int* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int v = nodes[i];
    int pmin = n;
    for (int p = rp[v]; p < rp[v + 1]; ++p) {
        const int u = ci[p];
        if (level[u] == L - 1) {
            const int q = pos[u];
            pmin = q < pmin ? q : pmin;
        }
    }
    const int deg = rp[v + 1] - rp[v];
    key[i] = ((unsigned long long)pmin << 8) | (unsigned long long)(deg < 255 ? deg : 255);
    val[i] = v;
}

// pos[order[i]] = first + i for the m nodes just placed
__global__ __launch_bounds__(kBlock) void k_cm_place(int m, const int* __restrict__ order, int first,
                                                     int* __restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) pos[order[i]] = first + (int)i;
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
