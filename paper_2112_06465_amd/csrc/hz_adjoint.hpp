// Adjoint (backward) kernels of the helmz library.
//
// For x = A^{-1} b and a real loss L with real-pair gradient g = dL/dRe x +
// i dL/dIm x, the adjoint state lambda solves A^H lambda = g; then
// dL/db = lambda and dL/dA_ij = -lambda_i conj(x_j) on A's pattern.
//
// A^H is formed on the device in CSR (count, scan, scatter, per-row sort),
// deterministically: the scatter order is fixed afterwards by sorting each
// row by column index, and columns are unique.  When the caller asserts
// A = A^T (HZ_SYMMETRIC), A^H = conj(A) and the adjoint solve is the forward
// solve on conjugated data: A conj(lambda) = conj(g).
#pragma once

#include "hz_kernels.hpp"

namespace hz {

// counts[col_p + 1] += 1 for every entry (integer atomics: exact)
__global__ __launch_bounds__(kBlock) void k_tr_count(int64_t nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[ci[p] + 1], 1);
}

// In-place inclusive scan of a[0..m) with one block: every thread scans a
// contiguous segment sequentially, segment totals are scanned in LDS, then
// added back.  Used once per adjoint set-up.
__global__ __launch_bounds__(1024) void k_scan_1block(int m, int* __restrict__ a) {
    __shared__ int tot[1024];
    const int t = threadIdx.x;
    const int seg = (m + 1023) / 1024;
    const int64_t lo = (int64_t)t * seg;
    const int64_t hi = lo + seg < m ? lo + seg : m;
    int s = 0;
    for (int64_t i = lo; i < hi; ++i) {
        s += a[i];
        a[i] = s;
    }
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int v = tot[k];
            tot[k] = run;
            run += v;
        }
    }
    __syncthreads();
    const int off = tot[t];
    for (int64_t i = lo; i < hi; ++i) a[i] += off;
}

// scatter (i, j, a) -> row j of A^H with value conj(a); fill[] starts as a copy of t_row_ptr
__global__ __launch_bounds__(kBlock) void k_tr_scatter(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double2* __restrict__ v, int* __restrict__ fill,
                                                       int* __restrict__ tci, double2* __restrict__ tv) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int q = atomicAdd(&fill[ci[p]], 1);
        tci[q] = (int)i;
        const double2 a = v[p];
        tv[q] = mk<double>(a.x, -a.y);
    }
}

// scatter entry p = (i, j) to row j of the transpose as column i, recording
// its source index p (the values of several systems are gathered by it later)
__global__ __launch_bounds__(kBlock) void k_tr_scatter_idx(int n, const int* __restrict__ rp,
                                                           const int* __restrict__ ci, int* __restrict__ fill,
                                                           int* __restrict__ tci, int* __restrict__ tsrc) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int q = atomicAdd(&fill[ci[p]], 1);
        tci[q] = (int)i;
        tsrc[q] = p;
    }
}

// sort each row of a CSR matrix by column, carrying a payload per entry (the
// values, or source entry indices); insertion sort, rows are short.  Used for
// the transpose and for P A P^T.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_row_sort(int n, const int* __restrict__ trp, int* __restrict__ tci,
                                                    V* __restrict__ tv) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int lo = trp[j], hi = trp[j + 1];
    for (int q = lo + 1; q < hi; ++q) {
        const int c = tci[q];
        const V a = tv[q];
        int k = q - 1;
        while (k >= lo && tci[k] > c) {
            tci[k + 1] = tci[k];
            tv[k + 1] = tv[k];
            --k;
        }
        tci[k + 1] = c;
        tv[k + 1] = a;
    }
}

// out = conj(in); in and out may be the same array
__global__ __launch_bounds__(kBlock) void k_conj(int n, const double2* in, double2* out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double2 a = in[i];
        out[i] = mk<double>(a.x, -a.y);
    }
}

// grad_vals[p] = -lambda_i conj(x_{col p}) for the entries p of row i (L lanes per row)
template <int L>
__global__ __launch_bounds__(kBlock) void k_grad_vals(int n, Geom geo, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const double2* __restrict__ lam,
                                                      const double2* __restrict__ x, double2* __restrict__ gv) {
    constexpr int RPS = kBlock / L;
    const Rows rw = rows_of_block(n, geo).rw;
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    for (int64_t row = rw.x0 + (int64_t)rw.k * RPS + g; row < rw.x1; row += (int64_t)rw.K * RPS) {
        const double2 l = lam[row];
        for (int p = rp[row] + lane; p < rp[row + 1]; p += L) {
            const double2 xv = x[ci[p]];
            // -(l * conj(xv))
            gv[p] = mk<double>(-__builtin_fma(l.x, xv.x, l.y * xv.y), -__builtin_fma(l.y, xv.x, -l.x * xv.y));
        }
    }
}

}  // namespace hz
