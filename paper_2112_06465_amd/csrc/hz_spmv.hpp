// Standalone row products y = A x (csr_zspmv, csr_cspmv, csr_zspmv_rect).
//
// The solver kernels fuse their row products with Krylov updates and block
// reductions (1024-thread blocks, at most 512 of them, so that every block can
// sum all partials).  A product on its own has no reduction, so it runs on
// 256-thread blocks, up to 16 per CU, in one of two forms that the autotuner
// picks per matrix:
//
// * pipelined vector rows (k_spmv_pipe): L lanes per row, U entries per lane
//   in the first batch.  The loop is unrolled twice with two register sets:
//   while the x gathers of the current tile are in flight, the (column,
//   value) loads of the next tile and the row_ptr loads of the tile after it
//   are already issued.  Every load is unconditional (indices clamped into
//   range, the results masked afterwards), so the hardware wait counters can
//   be waited on exactly, without a full drain at each step.
// * block tiles (k_spmv_tile): a tile of kTileRows rows whose entries are
//   loaded by the whole block contiguously (thread t takes entries e0 + t,
//   e0 + t + 256, ...), multiplied by the gathered x and written to LDS; then
//   kTileLanes threads per row sum the row's products out of LDS.  A tile
//   with more than kTileCap entries is done as vector rows instead.  Its
//   matrix loads are straight-line (clamped into the tile, masked after) and
//   streaming (ld_mat): each instruction reads 256 consecutive entries, whole
//   cache lines.  Up to kSpMaxGrid tiles, every tile gets a block; beyond,
//   kSpTileGrid blocks loop over the tiles (fewer concurrent streams measured
//   faster from HBM: 80 against 83 us on a 409 MB product).  The
//   results do not go to y tile by tile: a block keeps those of up to kHold
//   tiles in LDS and writes them in one pass when the ring is full and at its
//   end.  On this architecture one in-order counter tracks loads and stores,
//   so a store issued at the end of a tile made the next tile's first wait for
//   its loads also wait for the store to complete; with the ring a block's
//   stores hold up its loads once per kHold tiles (on the cabin's 409 MB
//   product, 19 tiles per block: 81 against 71-74 us).  With one tile per
//   block (fewer than kSpMaxGrid tiles) k_spmv_tile1 stores directly and
//   keeps the LDS, and with it the resident blocks, of the form without ring.
//
// Row ownership is that of the other kernels (XCD groups, tiles dealt out
// within a group), with the form's own tile height.  Summation order is fixed
// by the form and its lane count, so results are bitwise reproducible.
#pragma once

#include "hz_kernels.hpp"

namespace hz {

constexpr int kSpBlock = 256;                     // threads per block
constexpr int kSpMaxGrid = 4096;                  // blocks: 16 per CU
constexpr int kTileRows = 64;                     // rows per tile of the block form
constexpr int kTileLanes = kSpBlock / kTileRows;  // threads per row in its reduction
constexpr int kTilePer = 4;                       // entries per thread per tile
constexpr int kTileCap = kSpBlock * kTilePer;     // entries per tile held in LDS
constexpr int kSpTileGrid = 1024;                 // blocks of the tile form beyond kSpMaxGrid tiles
constexpr int kHold = 20;                         // tiles whose results a block holds in LDS (20 KB)

template <typename T> struct SpArgs {
    int n;    // rows
    int nnz;  // >= 1
    Geom geo;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const cx<T>* __restrict__ vals;
    const cx<T>* __restrict__ x;  // at least one element
    cx<T>* __restrict__ y;
    const int* __restrict__ yperm = nullptr;  // tile form: row r's result goes to y[yperm[r]] when set
};

template <typename T, int L, int U>
__global__ __launch_bounds__(kSpBlock) void k_spmv_pipe(const SpArgs<T> a) {
    constexpr int RPS = kSpBlock / L;
    const RowRange rr = rows_of_block(a.n, a.geo);
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    const int64_t first = rr.rw.x0 + (int64_t)rr.rw.k * RPS, step = (int64_t)rr.rw.K * RPS, r1 = rr.rw.x1;
    const int* __restrict__ rp = a.row_ptr;
    const int* __restrict__ ci = a.col_idx;
    const cx<T>* __restrict__ vals = a.vals;
    const cx<T>* __restrict__ x = a.x;
    const unsigned nnz = (unsigned)a.nnz;
    // entry range of row r (empty past the group's last row); loads stay in [0, n]
    auto bounds = [&](int64_t r, int& b, int& e) {
        const int64_t rc = r < r1 ? r : r1;
        const int b0 = rp[rc], e0 = rp[rc + 1 <= r1 ? rc + 1 : r1];
        b = r < r1 ? b0 : 0;
        e = r < r1 ? e0 : 0;
    };
    // first batch of a row: entry beg + lane + u L for u < U; col -1 marks an empty slot
    auto batch = [&](int b, int e, int (&c)[U], cx<T> (&v)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned p = (unsigned)b + (unsigned)(lane + u * L);
            const unsigned pc = p < nnz ? p : nnz - 1;
            const int cv = ci[pc];
            v[u] = vals[pc];
            c[u] = p < (unsigned)e ? cv : -1;
        }
    };
    // row `row` with entries [b, e) and first batch c/v; issues the next tile's batch
    // (entries [nb, ne) into c2/v2) and the row bounds two tiles ahead (into nnb/nne)
    auto one = [&](int64_t row, int b, int e, const int (&c)[U], const cx<T> (&v)[U], int nb, int ne, int (&c2)[U],
                   cx<T> (&v2)[U], int& nnb, int& nne) {
        cx<T> o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) o[u] = x[c[u] >= 0 ? c[u] : 0];
        batch(nb, ne, c2, v2);
        bounds(row + 2 * step, nnb, nne);
        cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const cx<T> f = cfma<T>(v[u], o[u], acc);
            const bool ok = c[u] >= 0;
            acc.x = ok ? f.x : acc.x;
            acc.y = ok ? f.y : acc.y;
        }
        if (e - b > L * U) {  // the rest of a long row, unpipelined
            const cx<T> rest = row_partial<T, L, U>(b + L * U, e, lane, ci, vals, [x](int cc) { return x[cc]; });
            acc.x += rest.x;
            acc.y += rest.y;
        }
        acc.x = group_sum<L>(acc.x);
        acc.y = group_sum<L>(acc.y);
        if (row < r1 && lane == 0) a.y[row] = acc;
    };
    int64_t row = first + g;
    int b0, e0, b1, e1;
    bounds(row, b0, e0);
    bounds(row + step, b1, e1);
    int c0[U], c1[U];
    cx<T> v0[U], v1[U];
    batch(b0, e0, c0, v0);
    for (int64_t base = first; base < r1; base += 2 * step) {
        one(row, b0, e0, c0, v0, b1, e1, c1, v1, b0, e0);
        if (base + step >= r1) break;
        one(row + step, b1, e1, c1, v1, b0, e0, c0, v0, b1, e1);
        row += 2 * step;
    }
}

// The tile loop of a block over the 64-row tiles that `rw` describes (the
// block is the rw.k-th of rw.K taking the tiles of [x0, x1) in turn).  op(col)
// is the gathered operand.  Each row's total goes to tail(row, total,
// pre(row)) as soon as the tile is summed (pre: an operand per row, loaded
// with the tile's matrix entries; NoPre: no load) and to put(row, total),
// which stores it.  HOLD > 1: put runs when an LDS ring of HOLD tiles' totals
// is flushed (full, or at the end); HOLD = 1: at once (one tile per block,
// where a ring would only cost LDS, and so resident blocks).  A flush issues
// stores only, so its stores hold up the next tile's loads once per HOLD
// tiles and the last flush leaves nothing to wait for.  A tile of empty rows
// loads nothing; every branch is uniform across the block.
template <typename T, int HOLD, typename Op, typename Pre, typename Tail, typename Put>
__device__ __forceinline__ void tile_loop(const Rows& rw, const int* __restrict__ rp, const int* __restrict__ ci,
                                          const cx<T>* __restrict__ vals, Op op, Pre pre, Tail tail, Put put) {
    constexpr int L = kTileLanes;
    __shared__ cx<T> prod[kTileCap];
    __shared__ cx<T> held[HOLD > 1 ? HOLD * kTileRows : 1];  // totals of the block's last tiles, by tile
    const int t = threadIdx.x, g = t / L, lane = t % L;
    const int64_t first = rw.x0 + (int64_t)rw.k * kTileRows, step = (int64_t)rw.K * kTileRows;
    const int64_t r1 = rw.x1;
    // the `count` held tiles starting at the block's tile `base` (every thread; uniform)
    auto flush = [&](int64_t base, int count) {
        __syncthreads();  // the held totals are written
        for (int q = t; q < count * kTileRows; q += kSpBlock) {
            const int64_t row = first + (base + q / kTileRows) * step + q % kTileRows;
            if (row < r1) put(row, held[q]);
        }
        __syncthreads();  // the ring may be refilled
    };
    int64_t tile = 0;                                        // the block's tile counter
    for (int64_t r0 = first; r0 < r1; r0 += step, ++tile) {  // uniform across the block
        const int64_t re = r0 + kTileRows < r1 ? r0 + kTileRows : r1;
        const int e0 = rp[r0], e1 = rp[re];
        const int64_t row = r0 + g;
        const int b = rp[row < re ? row : re], e = rp[row + 1 < re ? row + 1 : re];
        const auto w = pre(row < re ? row : re - 1);
        cx<T> acc = mk<T>(T(0), T(0));
        if (e1 > e0 && e1 - e0 <= kTileCap) {
            // straight-line streaming loads: entry e0 + t + k kSpBlock, clamped into the tile
            const int last = e1 - 1;
            int c[kTilePer];
            cx<T> v[kTilePer], o[kTilePer];
#pragma unroll
            for (int k = 0; k < kTilePer; ++k) {
                const int p = e0 + t + k * kSpBlock;
                c[k] = ld_mat(ci + (p < last ? p : last));
            }
#pragma unroll
            for (int k = 0; k < kTilePer; ++k) {
                const int p = e0 + t + k * kSpBlock;
                v[k] = ld_mat(vals + (p < last ? p : last));
            }
#pragma unroll
            for (int k = 0; k < kTilePer; ++k) o[k] = op(c[k]);
#pragma unroll
            for (int k = 0; k < kTilePer; ++k) {
                const bool ok = e0 + t + k * kSpBlock < e1;
                const cx<T> pr = cmul<T>(v[k], o[k]);
                prod[t + k * kSpBlock] = mk<T>(ok ? pr.x : T(0), ok ? pr.y : T(0));
            }
            __syncthreads();
            for (int q = b - e0 + lane; q < e - e0; q += L) {
                const cx<T> pv = prod[q];
                acc.x += pv.x;
                acc.y += pv.y;
            }
            __syncthreads();
        } else if (e1 > e0 && row < re) {
            acc = row_partial<T, L, 1>(b, e, lane, ci, vals, op);
        }
        acc.x = group_sum<L>(acc.x);
        acc.y = group_sum<L>(acc.y);
        if (row < re && lane == 0) tail(row, acc, w);
        if constexpr (HOLD > 1) {
            const int slot = (int)(tile % HOLD);
            if (lane == 0) held[slot * kTileRows + g] = acc;  // (rows past the range are skipped by the flush)
            if (slot == HOLD - 1) flush(tile - (HOLD - 1), HOLD);
        } else if (row < re && lane == 0) {
            put(row, acc);
        }
    }
    if constexpr (HOLD > 1) {
        if (tile % HOLD != 0) flush(tile - tile % HOLD, (int)(tile % HOLD));
    }
}

// No per-row work besides the store.
struct NoTail {
    template <typename A, typename W> __device__ void operator()(int64_t, A, W) const {}
};

template <typename T, int HOLD>
__device__ __forceinline__ void spmv_tiles(const SpArgs<T>& a) {
    const RowRange rr = rows_of_block(a.n, a.geo);
    const cx<T>* __restrict__ x = a.x;
    cx<T>* __restrict__ y = a.y;
    const int* __restrict__ yperm = a.yperm;
    tile_loop<T, HOLD>(rr.rw, a.row_ptr, a.col_idx, a.vals, [x](int c) { return x[c]; }, NoPre{}, NoTail{},
                       [=](int64_t row, cx<T> acc) { y[yperm != nullptr ? yperm[row] : row] = acc; });
}

template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_spmv_tile(const SpArgs<T> a) {
    spmv_tiles<T, kHold>(a);
}

template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_spmv_tile1(const SpArgs<T> a) {
    spmv_tiles<T, 1>(a);
}

}  // namespace hz
