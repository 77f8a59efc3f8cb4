// The two row products of the gather-light BiCGStab iteration (Section 7:
// v = A p with <rhat, v>, and t = A s with <t, s> and ||t||^2) in the
// standalone product's tile form, for one large system (BiCGstab(l)'s two
// products, with the same structure, are in hz_bicgstabl.hpp).
//
// The solver's other kernels run 1024-thread blocks, at most kMaxGrid of
// them, and under their 64-VGPR budget a product could not hold its results
// back without spilling; its stores then sat in front of the next tile's
// loads (one in-order counter tracks both).  These kernels run each logical
// block of the solver's map as F = sol_subs(G) blocks of kSpBlock threads
// (half the waves per CU at most, twice the registers per wave) through
// tile_loop with its LDS ring: the epilogue operand of each row (rhat or s) is loaded with the
// tile's matrix entries and the row's terms go into the block's dot products
// as soon as the tile is summed, while the totals v (or t) are held for kHold
// tiles and stored when the ring is flushed.  Sub-block j of logical block lb
// takes 64-row tiles k' = F k + j of its group's rows (K' = F K), and writes
// its partials to slot F lb + j; the region's readers sum F slots per block
// (BicgArgs::pf = F), and the S kernel, which writes the region's first
// component with the logical blocks, fills the extra slots with zeros.  Sums are taken in a fixed order: results are bitwise
// reproducible.
#pragma once

#include "hz_spmv.hpp"

namespace hz {

constexpr int kSolSlots = 1024;  // partial slots per component that the sub-blocks of a launch may take

// Product blocks per logical block of a map of G blocks: enough for about
// kSolSlots blocks (four per CU, the residency that the tile loop's 36 KB of
// LDS allows), at least 2 and at most 4, and F G <= max(2 G, kSolSlots).
__host__ __device__ constexpr int sol_subs(int G) {
    const int f = G > 0 ? kSolSlots / G : 4;
    return f < 2 ? 2 : (f > 4 ? 4 : f);
}

struct SubBlock {
    int ls, sys;
    Rows rw;
};
// Sub-block of a launch of F G blocks over the solver map `bmap` of G blocks.
__device__ __forceinline__ SubBlock sub_block_of(const BlockMap* bmap, int G, int F) {
    SubBlock q;
    q.ls = logical_block(blockIdx.x, F * G);
    const BlockMap m = bmap[q.ls / F];
    q.sys = m.sys;
    q.rw.x0 = m.x0;
    q.rw.x1 = m.x1;
    q.rw.k = F * m.k + q.ls % F;
    q.rw.K = F * m.K;
    return q;
}
template <typename T> __device__ __forceinline__ SubBlock sub_block(const BicgArgs<T>& a) {
    return sub_block_of(a.bmap, a.G, a.pf);
}

template <int K>
__device__ __forceinline__ void store_sub_partials(double* __restrict__ part, int stride, int ls, double (&e)[K]) {
    block_sum<K, kSpBlock>(e);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[k * stride + ls] = e[k];
    }
}

template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_bicg_A1t(const BicgArgs<T> a) {
    const SubBlock q = sub_block(a);
    if (q.sys < 0) return;
    const SolverScal* sc = a.sc + q.sys;
    if (sc->done || sc->pending) return;
    const int it = sc->cur;
    const cx<T>* __restrict__ p = a.p[it & 1];
    cx<T>* __restrict__ v = a.v[it & 1];
    const cx<T>* __restrict__ rh = a.rh;
    double e[2] = {0.0, 0.0};
    tile_loop<T, kHold>(
        q.rw, a.row_ptr, a.col_idx, a.vals, [p](int c) { return p[c]; }, [rh](int64_t row) { return rh[row]; },
        [&](int64_t, cx<T> acc, cx<T> w) {
            const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        },
        [v](int64_t row, cx<T> acc) { v[row] = acc; });
    store_sub_partials<2>(a.part + kPartA * a.stride, a.stride, q.ls, e);
}

template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_bicg_B1t(const BicgArgs<T> a) {
    const SubBlock q = sub_block(a);
    if (q.sys < 0) return;
    if (a.sc[q.sys].done) return;
    const cx<T>* __restrict__ sv = a.s;
    cx<T>* __restrict__ tv = a.t;
    double e[3] = {0.0, 0.0, 0.0};
    tile_loop<T, kHold>(
        q.rw, a.row_ptr, a.col_idx, a.vals, [sv](int c) { return sv[c]; }, [sv](int64_t row) { return sv[row]; },
        [&](int64_t, cx<T> acc, cx<T> s) {
            const double2 c = cdotacc(acc.x, acc.y, s.x, s.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
            e[2] = __builtin_fma((double)acc.x, (double)acc.x, e[2]);
            e[2] = __builtin_fma((double)acc.y, (double)acc.y, e[2]);
        },
        [tv](int64_t row, cx<T> acc) { tv[row] = acc; });
    store_sub_partials<3>(a.part + (kPartB + 1) * a.stride, a.stride, q.ls, e);
}

}  // namespace hz
