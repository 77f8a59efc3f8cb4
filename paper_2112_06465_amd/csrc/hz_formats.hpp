// Storage formats beside CSR: ELL / HYB and SELL-C-sigma (Section 3.2 lists
// COO, ELL and HYB as the alternatives to its CSR; SELL-C-sigma is Kreutzer
// et al.'s sliced ELL, with t lanes per row as in Anzt et al.'s SELL-P).
//
// ELL of width K: entry k of row i at k*n + i, padding column -1, value 0.
// HYB: ELL of width K plus the rest of each row as COO triplets in CSR order.
// SELL-C-sigma, t lanes per row: sorted position p holds row perm[p] (rows
// sorted by decreasing length within windows of sigma rows, ties in row
// order), chunk c = p / C, row r = p % C, chunk width w_c (the chunk's
// longest row rounded up to a multiple of t), chunk_ptr[c + 1] -
// chunk_ptr[c] = C w_c, entry k at chunk_ptr[c] + (k / t) C t + r t + k % t.
//
// Products run one thread per row (t lanes per row for SELL, reduced by
// cross-lane shuffles); the loads of a step are unconditional (padding reads
// x of the thread's own row and is zeroed by selects), so consecutive
// threads' slots are consecutive in memory and the loads of a row stream.
#pragma once

#include "hz_kernels.hpp"

namespace hz {

constexpr int kFmtBlock = 256;

__device__ __forceinline__ int64_t fmt_thread(int G) {
    return (int64_t)logical_block(blockIdx.x, G) * kFmtBlock + threadIdx.x;
}

// len_i of every row (as sort keys)
__global__ __launch_bounds__(kFmtBlock) void k_fmt_len(int n, const int* __restrict__ rp, unsigned* __restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (i < n) len[i] = (unsigned)(rp[i + 1] - rp[i]);
}

// From the lengths sorted in decreasing order: the longest row and the HYB
// width (the ceil(n/3)-th longest length: the largest K that at least a
// third of the rows reach).
__global__ void k_fmt_stats(int n, const unsigned* __restrict__ sorted, int* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    out[0] = (int)sorted[0];
    out[1] = (int)sorted[(n + 2) / 3 - 1];
}

// rem_i = max(0, len_i - K) for i < n, rem_n = 0 (scanned into the COO offsets)
__global__ __launch_bounds__(kFmtBlock) void k_hyb_rem(int n, const int* __restrict__ rp, int K, int* __restrict__ rem) {
    const int64_t i = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (i > n) return;
    const int len = i < n ? rp[i + 1] - rp[i] : 0;
    rem[i] = len > K ? len - K : 0;
}

// One thread per row: its ELL slots (entries or padding), then its COO entries.
__global__ __launch_bounds__(kFmtBlock) void k_hyb_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const double2* __restrict__ vals, int K,
                                                        const int* __restrict__ off, int* __restrict__ ell_col,
                                                        double2* __restrict__ ell_val, int* __restrict__ coo_row,
                                                        int* __restrict__ coo_col, double2* __restrict__ coo_val) {
    const int64_t i = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (i >= n) return;
    const int lo = rp[i], len = rp[i + 1] - lo;
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)k * n + i;
        if (k < len) {
            ell_col[q] = ci[lo + k];
            ell_val[q] = vals[lo + k];
        } else {
            ell_col[q] = -1;
            ell_val[q] = mk<double>(0.0, 0.0);
        }
    }
    for (int k = K; k < len; ++k) {
        const int e = off[i] + (k - K);
        coo_row[e] = (int)i;
        coo_col[e] = ci[lo + k];
        coo_val[e] = vals[lo + k];
    }
}

// y_i = sum over row i's ELL slots; U slots loaded before their products.
template <int U>
__global__ __launch_bounds__(kFmtBlock) void k_ell_spmv(int n, int K, int G, const int* __restrict__ col,
                                                        const double2* __restrict__ val,
                                                        const double2* __restrict__ x, double2* __restrict__ y) {
    const int64_t i = fmt_thread(G);
    if (i >= n) return;
    double ax = 0.0, ay = 0.0;
    int k = 0;
    for (; k + U <= K; k += U) {
        int c[U];
        double2 v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = (int64_t)(k + u) * n + i;
            c[u] = col[q];
            v[u] = val[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u] < 0 ? i : c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool pad = c[u] < 0;
            const double vx = pad ? 0.0 : v[u].x, vy = pad ? 0.0 : v[u].y;
            ax = __builtin_fma(vx, xv[u].x, ax);
            ax = __builtin_fma(-vy, xv[u].y, ax);
            ay = __builtin_fma(vx, xv[u].y, ay);
            ay = __builtin_fma(vy, xv[u].x, ay);
        }
    }
    for (; k < K; ++k) {
        const int64_t q = (int64_t)k * n + i;
        const int c = col[q];
        const double2 v = val[q], xv = x[c < 0 ? i : c];
        const bool pad = c < 0;
        const double vx = pad ? 0.0 : v.x, vy = pad ? 0.0 : v.y;
        ax = __builtin_fma(vx, xv.x, ax);
        ax = __builtin_fma(-vy, xv.y, ax);
        ay = __builtin_fma(vx, xv.y, ay);
        ay = __builtin_fma(vy, xv.x, ay);
    }
    y[i] = mk<double>(ax, ay);
}

// Rows of at most U slots (1 <= K <= U): all of a thread's slot loads in one
// straight-line batch (slot indices clamped to K - 1, the extra ones
// zeroed), so the whole row is in flight at once.  One thread per row leaves
// few waves per SIMD on these matrices, so the loads in flight per thread
// set the product's bandwidth.
template <int U>
__global__ __launch_bounds__(kFmtBlock) void k_ell_spmv_full(int n, int K, int G, const int* __restrict__ col,
                                                             const double2* __restrict__ val,
                                                             const double2* __restrict__ x,
                                                             double2* __restrict__ y) {
    const int64_t i = fmt_thread(G);
    if (i >= n) return;
    int c[U];
    double2 v[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t q = (int64_t)(u < K ? u : K - 1) * n + i;
        c[u] = col[q];
        v[u] = val[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u] < 0 ? i : c[u]];
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool pad = u >= K || c[u] < 0;
        const double vx = pad ? 0.0 : v[u].x, vy = pad ? 0.0 : v[u].y;
        ax = __builtin_fma(vx, xv[u].x, ax);
        ax = __builtin_fma(-vy, xv[u].y, ax);
        ay = __builtin_fma(vx, xv[u].y, ay);
        ay = __builtin_fma(vy, xv[u].x, ay);
    }
    y[i] = mk<double>(ax, ay);
}

// COO part of a HYB product: the thread of a row's first COO entry sums the
// row's COO entries in order and adds them to y (one writer per row).
__global__ __launch_bounds__(kFmtBlock) void k_coo_add(int m, const int* __restrict__ row, const int* __restrict__ col,
                                                       const double2* __restrict__ val,
                                                       const double2* __restrict__ x, double2* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (e >= m) return;
    const int r = row[e];
    if (e > 0 && row[e - 1] == r) return;
    double ax = 0.0, ay = 0.0;
    for (int64_t q = e; q < m && row[q] == r; ++q) {
        const double2 v = val[q], xv = x[col[q]];
        ax = __builtin_fma(v.x, xv.x, ax);
        ax = __builtin_fma(-v.y, xv.y, ax);
        ay = __builtin_fma(v.x, xv.y, ay);
        ay = __builtin_fma(v.y, xv.x, ay);
    }
    const double2 yv = y[r];
    y[r] = mk<double>(yv.x + ax, yv.y + ay);
}

// ------------------------------------------------------------------ SELL-C-sigma

// Sort keys: window (i / sigma) above, 2^32 - 1 - len_i below, so an
// ascending stable sort orders each window by decreasing length, ties by row.
__global__ __launch_bounds__(kFmtBlock) void k_sell_keys(int n, const int* __restrict__ rp, int sigma,
                                                         unsigned long long* __restrict__ key, int* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (i >= n) return;
    const unsigned len = (unsigned)(rp[i + 1] - rp[i]);
    key[i] = ((unsigned long long)(i / sigma) << 32) | (unsigned long long)(0xffffffffu - len);
    idx[i] = (int)i;
}

__global__ __launch_bounds__(kFmtBlock) void k_iota(int n, int* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (i < n) perm[i] = (int)i;
}

// cw[c] = C w_c for c < nch, cw[nch] = 0 (scanned into chunk_ptr)
__global__ __launch_bounds__(kFmtBlock) void k_sell_widths(int n, int nch, int C, int t, const int* __restrict__ rp,
                                                           const int* __restrict__ perm,
                                                           long long* __restrict__ cw) {
    const int64_t c = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (c > nch) return;
    if (c == nch) {
        cw[c] = 0;
        return;
    }
    int longest = 0;
    const int64_t p1 = (c + 1) * C < n ? (c + 1) * C : n;
    for (int64_t p = c * C; p < p1; ++p) {
        const int row = perm[p];
        const int len = rp[row + 1] - rp[row];
        longest = len > longest ? len : longest;
    }
    const int w = (longest + t - 1) / t * t;
    cw[c] = (long long)C * w;
}

// One thread per sorted position (padding rows of the last chunk included):
// its row's entries and padding.  Any inconsistency of perm / chunk_ptr with
// the matrix or the capacity sets *err and writes nothing for that row.
__global__ __launch_bounds__(kFmtBlock) void k_sell_fill(int n, int nch, int C, int t, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double2* __restrict__ vals,
                                                         const int* __restrict__ perm,
                                                         const long long* __restrict__ chunk_ptr, long long slots,
                                                         int* __restrict__ col, double2* __restrict__ val, int* err) {
    const int64_t p = (int64_t)blockIdx.x * kFmtBlock + threadIdx.x;
    if (p >= (int64_t)nch * C) return;
    const int64_t c = p / C, r = p % C;
    const long long lo = chunk_ptr[c], hi = chunk_ptr[c + 1];
    if (lo < 0 || hi > slots || hi < lo || (hi - lo) % C != 0 || ((hi - lo) / C) % t != 0) {
        *err = 1;
        return;
    }
    const int w = (int)((hi - lo) / C);
    int row = -1, beg = 0, len = 0;
    if (p < n) {
        row = perm[p];
        if (row < 0 || row >= n) {
            *err = 1;
            return;
        }
        beg = rp[row];
        len = rp[row + 1] - beg;
        if (len > w) {
            *err = 1;
            return;
        }
    }
    for (int k = 0; k < w; ++k) {
        const int64_t q = lo + (int64_t)(k / t) * C * t + r * t + (k % t);
        if (k < len) {
            col[q] = ci[beg + k];
            val[q] = vals[beg + k];
        } else {
            col[q] = -1;
            val[q] = mk<double>(0.0, 0.0);
        }
    }
}

// y[perm[p]] = sum over sorted position p's slots; T lanes per row (lane j
// takes the slots k = j, j + T, ...), U slot loads in flight per lane.
template <int T, int U>
__global__ __launch_bounds__(kFmtBlock) void k_sell_spmv(int n, int nch, int C, int G, const int* __restrict__ perm,
                                                         const long long* __restrict__ chunk_ptr,
                                                         const int* __restrict__ col, const double2* __restrict__ val,
                                                         const double2* __restrict__ x, double2* __restrict__ y) {
    const int64_t g = fmt_thread(G);
    const int64_t p = g / T;
    const int j = (int)(g % T);
    if (p >= (int64_t)nch * C) return;  // the T lanes of a row leave together
    const int64_t c = p / C, r = p % C;
    const long long lo = chunk_ptr[c];
    const int steps = (int)((chunk_ptr[c + 1] - lo) / C) / T;
    const int64_t base = lo + r * T + j, stride = (int64_t)C * T;
    const int64_t self = p < n ? p : 0;  // padding slots read x of a fixed nearby entry
    double ax = 0.0, ay = 0.0;
    int s = 0;
    for (; s + U <= steps; s += U) {
        int cc[U];
        double2 v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = base + (int64_t)(s + u) * stride;
            cc[u] = col[q];
            v[u] = val[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[cc[u] < 0 ? self : cc[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool pad = cc[u] < 0;
            const double vx = pad ? 0.0 : v[u].x, vy = pad ? 0.0 : v[u].y;
            ax = __builtin_fma(vx, xv[u].x, ax);
            ax = __builtin_fma(-vy, xv[u].y, ax);
            ay = __builtin_fma(vx, xv[u].y, ay);
            ay = __builtin_fma(vy, xv[u].x, ay);
        }
    }
    for (; s < steps; ++s) {
        const int64_t q = base + (int64_t)s * stride;
        const int ci = col[q];
        const double2 v = val[q], xv = x[ci < 0 ? self : ci];
        const bool pad = ci < 0;
        const double vx = pad ? 0.0 : v.x, vy = pad ? 0.0 : v.y;
        ax = __builtin_fma(vx, xv.x, ax);
        ax = __builtin_fma(-vy, xv.y, ax);
        ay = __builtin_fma(vx, xv.y, ay);
        ay = __builtin_fma(vy, xv.x, ay);
    }
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) {
        ax += __shfl_xor(ax, o, T);
        ay += __shfl_xor(ay, o, T);
    }
    if (j == 0 && p < n) y[perm[p]] = mk<double>(ax, ay);
}

}  // namespace hz
