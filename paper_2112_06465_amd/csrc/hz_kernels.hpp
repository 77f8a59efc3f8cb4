// Device kernels of the helmz library (gfx950 / CDNA4, wave64).
//
// Reductions: every reducing kernel writes one fixed-order partial per block
// (component-major, stride kMaxGrid).  The kernel that needs the total sums
// the partials itself, redundantly in every block and in a fixed order, so
// all blocks hold bitwise the same scalar and no single-block finaliser
// kernel sits between two streaming kernels.  No floating-point atomics:
// results are bitwise reproducible run to run.
//
// Row ownership: a launch of G blocks splits the rows into G contiguous
// chunks.  Hardware dispatches block b to XCD (b mod 8); block b works on
// logical chunk (b mod 8) * (G/8) + b/8, so each XCD owns one contiguous
// eighth of the rows.  The x-gathers of a banded FE matrix then stay inside
// that XCD's L2, and every kernel of a solve maps the same rows to the same
// XCD.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace hz {

constexpr int kWave = 64;
constexpr int kXcd = 8;
constexpr int kBlock = 1024;   // threads per block (16 waves)
constexpr int kMaxGrid = 512;  // bound on blocks (= partials) of a reducing launch: 2 blocks per CU
#define HZ_STREAM_BOUNDS __launch_bounds__(1024, 8)  // 8 waves per SIMD (two blocks per CU): <= 64 VGPRs

// partial-sum regions (component index; component c lives at part[c * kMaxGrid + block])
constexpr int kPartA = 0;  // <rhat, v>                      (2)
constexpr int kPartB = 2;  // ||s||^2, <t, s>, ||t||^2         (4)
constexpr int kPartC = 6;  // <rhat, r>, ||r||^2               (3)
constexpr int kPartI = 9;  // ||b||^2 / residual norms          (1)
constexpr int kParts = 10;

// ------------------------------------------------------------------ complex

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cx = typename cplx_of<T>::type;

template <typename T> __device__ __forceinline__ cx<T> mk(T re, T im) {
    cx<T> z;
    z.x = re;
    z.y = im;
    return z;
}
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// c + a b
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
    c.x = fmaT(a.x, b.x, c.x);
    c.x = fmaT(-a.y, b.y, c.x);
    c.y = fmaT(a.x, b.y, c.y);
    c.y = fmaT(a.y, b.x, c.y);
    return c;
}
// a b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return mk<T>(fmaT(a.x, b.x, -a.y * b.y), fmaT(a.x, b.y, a.y * b.x));
}
// c + conj(a) b, accumulated in double
__device__ __forceinline__ double2 cdotacc(double ar, double ai, double br, double bi, double2 c) {
    c.x = __builtin_fma(ar, br, c.x);
    c.x = __builtin_fma(ai, bi, c.x);
    c.y = __builtin_fma(ar, bi, c.y);
    c.y = __builtin_fma(-ai, br, c.y);
    return c;
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    double2 q;
    q.x = (a.x * b.x + a.y * b.y) / d;
    q.y = (a.y * b.x - a.x * b.y) / d;
    return q;
}
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    double2 q;
    q.x = a.x * b.x - a.y * b.y;
    q.y = a.x * b.y + a.y * b.x;
    return q;
}
__device__ __forceinline__ bool zfinite(double2 a) { return __builtin_isfinite(a.x) && __builtin_isfinite(a.y); }
__device__ __forceinline__ bool zzero(double2 a) { return a.x == 0.0 && a.y == 0.0; }
template <typename T> __device__ __forceinline__ cx<T> narrow(double2 a) { return mk<T>((T)a.x, (T)a.y); }

// Streaming (non-temporal) loads of matrix arrays, for kernels whose every
// load instruction covers whole cache lines of consecutive entries (the block
// tiles of the standalone product): the data is read once, and on this part
// such streaming loads sustain 5-10 % more HBM bandwidth than ordinary ones.
// Row-split accesses (L lanes per row, a line shared by neighbouring rows) and
// the solvers' products, whose matrix is re-read every iteration, measured
// slower with them and use ordinary loads.  HZ_STREAM_MATRIX=0 at build time
// makes these ordinary loads too.
#ifndef HZ_STREAM_MATRIX
#define HZ_STREAM_MATRIX 1
#endif
typedef double hz_d2v __attribute__((ext_vector_type(2)));
typedef float hz_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int ld_mat(const int* p) {
#if HZ_STREAM_MATRIX
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
__device__ __forceinline__ double2 ld_mat(const double2* p) {
#if HZ_STREAM_MATRIX
    const hz_d2v v = __builtin_nontemporal_load(reinterpret_cast<const hz_d2v*>(p));
    return mk<double>(v.x, v.y);
#else
    return *p;
#endif
}
__device__ __forceinline__ float2 ld_mat(const float2* p) {
#if HZ_STREAM_MATRIX
    const hz_f2v v = __builtin_nontemporal_load(reinterpret_cast<const hz_f2v*>(p));
    return mk<float>(v.x, v.y);
#else
    return *p;
#endif
}

// ------------------------------------------------------------------ lane exchange (DPP / ds_swizzle)

struct I2 {
    int lo, hi;
};

template <int CTRL> __device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int PAT> __device__ __forceinline__ int swz_i32(int v) { return __builtin_amdgcn_ds_swizzle(v, PAT); }

template <int CTRL> __device__ __forceinline__ double dpp(double v) {
    I2 w = __builtin_bit_cast(I2, v);
    w.lo = dpp_i32<CTRL>(w.lo);
    w.hi = dpp_i32<CTRL>(w.hi);
    return __builtin_bit_cast(double, w);
}
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, dpp_i32<CTRL>(__builtin_bit_cast(int, v)));
}
template <int PAT> __device__ __forceinline__ double swz(double v) {
    I2 w = __builtin_bit_cast(I2, v);
    w.lo = swz_i32<PAT>(w.lo);
    w.hi = swz_i32<PAT>(w.hi);
    return __builtin_bit_cast(double, w);
}
template <int PAT> __device__ __forceinline__ float swz(float v) {
    return __builtin_bit_cast(float, swz_i32<PAT>(__builtin_bit_cast(int, v)));
}

// DPP controls (gfx9 encoding)
constexpr int kQuadXor1 = 0xB1;     // quad_perm(1,0,3,2)
constexpr int kQuadXor2 = 0x4E;     // quad_perm(2,3,0,1)
constexpr int kHalfMirror = 0x141;  // lane i <-> 7-i inside each group of 8
constexpr int kMirror = 0x140;      // lane i <-> 15-i inside each row of 16
constexpr int kSwzXor16 = 0x401F;   // ds_swizzle bit mode: lane ^ 16 within 32

// Sum over aligned groups of L lanes; every lane of a group receives the same
// bitwise value (each step adds a value and its partner's, a + b == b + a).
// All 64 lanes must be active.
template <int L, typename T> __device__ __forceinline__ T group_sum(T v) {
    static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16 || L == 32 || L == 64, "L");
    if constexpr (L >= 2) v += dpp<kQuadXor1>(v);
    if constexpr (L >= 4) v += dpp<kQuadXor2>(v);
    if constexpr (L >= 8) v += dpp<kHalfMirror>(v);
    if constexpr (L >= 16) v += dpp<kMirror>(v);
    if constexpr (L >= 32) v += swz<kSwzXor16>(v);
    if constexpr (L >= 64) v += __shfl_xor(v, 32);
    return v;
}

// Block sum of K doubles over a block of NT threads; the result is valid in
// thread 0 only.  Waves are combined in a fixed order.  Safe to call
// repeatedly in one kernel.
template <int K, int NT = kBlock> __device__ __forceinline__ void block_sum(double (&v)[K]) {
    __shared__ double lds[NT / kWave][K];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = group_sum<64>(v[k]);
    __syncthreads();  // a previous call's reader is done with lds
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wid][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = lds[0][k];
            for (int w = 1; w < NT / kWave; ++w) s += lds[w][k];
            v[k] = s;
        }
    }
}

// Sum of K partial components (component k at part[k*kMaxGrid + g], g < G)
// in a fixed order, delivered to every thread of the block.
// (G <= kMaxGrid <= kBlock: one partial per thread, the K loads issued
// together; idle waves load nothing, as in sys_sum.)
template <int K> __device__ __forceinline__ void head_sum(const double* __restrict__ part, int G, double (&out)[K]) {
    static_assert(kMaxGrid <= kBlock, "one partial per thread");
    __shared__ double bc[K];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    if ((__builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~(kWave - 1)) < G) {
        const bool mine = t < G;
        const int g0 = mine ? t : G - 1;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double v = part[k * kMaxGrid + g0];
            out[k] = mine ? v : 0.0;
        }
    }
    block_sum<K>(out);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) bc[k] = out[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = bc[k];
}

// Store a block's K partials (thread 0 holds them after block_sum).
template <int K> __device__ __forceinline__ void store_partials(double* __restrict__ part, int lb, double (&e)[K]) {
    block_sum<K>(e);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[k * kMaxGrid + lb] = e[k];
    }
}

// ------------------------------------------------------------------ launch geometry

// Chunked row ownership of a launch (see the file comment).
struct Geom {
    int G;  // blocks: a multiple of 8 when there are at least 8
};

__device__ __forceinline__ int logical_block(int b, int G) {
    return (G % kXcd == 0) ? (b % kXcd) * (G / kXcd) + b / kXcd : b;
}

// The rows of a block.  The block is the k-th of the K blocks that share the
// row range [x0, x1) of its group and takes that range's tiles k, k + K,
// k + 2K, ... (a tile is kBlock/L rows in a row product, kBlock rows in an
// element-wise pass).  A launch of G >= 8 blocks has 8 groups, one per XCD,
// each owning an eighth of the rows; the K blocks of an XCD then advance
// through its range side by side, so the part of x their gathers touch at
// any time is a few tiles plus the matrix bandwidth, small enough for the
// XCD's L2 (with one contiguous chunk per block it would be K separate
// windows).  A system of a batch with its own chunk per block is K = 1.
struct Rows {
    int64_t x0, x1;
    int k, K;
};
__device__ __forceinline__ Rows group_rows(int n, int G, int lb) {
    Rows r;
    const int groups = (G % kXcd == 0) ? kXcd : 1;
    r.K = G / groups;
    const int x = lb / r.K;
    r.k = lb % r.K;
    r.x0 = (int64_t)n * x / groups;
    r.x1 = (int64_t)n * (x + 1) / groups;
    return r;
}

struct RowRange {
    int lb;
    Rows rw;
};
__device__ __forceinline__ RowRange rows_of_block(int n, Geom geo) {
    RowRange r;
    r.lb = logical_block(blockIdx.x, geo.G);
    r.rw = group_rows(n, geo.G, r.lb);
    return r;
}

// Element-wise pass over the rows of a block (tiles of kBlock rows).
#define HZ_FOR_ELEMS(i, rw) \
    for (int64_t i = (rw).x0 + (int64_t)(rw).k * kBlock + threadIdx.x; i < (rw).x1; i += (int64_t)(rw).K * kBlock)

// ------------------------------------------------------------------ row product (vector CSR)

// sum_p vals_p * op(col_p) over one row, computed by L lanes: lane l takes
// entries beg+l, beg+l+L, ...; each lane issues U (col, value) loads, then U
// operand gathers, then U complex FMAs, so U independent loads of each kind
// are in flight per lane.  The loads are straight-line: an entry past the
// row's end is read at the row's last entry (in bounds, since the loop runs
// only while base < end) and its product is dropped by selects on the
// accumulator, so no load is exec-masked (a masked load makes the compiler
// wait for every load in flight).  Returns the lane's partial (the caller
// sums the group).  Entry order per lane is sequential, so results are
// deterministic.
template <typename T, int L, int U, typename Op>
__device__ __forceinline__ cx<T> row_partial(int beg, int end, int lane, const int* __restrict__ ci,
                                             const cx<T>* __restrict__ vals, Op op) {
    cx<T> acc = mk<T>(T(0), T(0));
    for (int base = beg + lane; base < end; base += L * U) {
        int c[U];
        cx<T> a[U], o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = base + u * L < end ? base + u * L : end - 1;
            c[u] = ci[p];
            a[u] = vals[p];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) o[u] = op(c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = base + u * L < end;
            const cx<T> nx = cfma<T>(a[u], o[u], acc);
            acc.x = in ? nx.x : acc.x;
            acc.y = in ? nx.y : acc.y;
        }
    }
    return acc;
}

// Block-tile form of the row loop (the lane count L = 1 selects it): tiles
// of kSolTileRows rows; the block loads a tile's entries [rp[r0], rp[r0 +
// kSolTileRows]) contiguously (thread t takes entries e0 + t + k kBlock,
// straight-line, clamped into the tile), multiplies them by the gathered
// operand op(col), writes the products to LDS, and kSolTileLanes threads per
// row sum the row out of LDS in entry order; epi(row, total) runs in the
// first thread of each row.  Each load instruction reads kBlock consecutive
// entries, whole cache lines, where the vector form reads a row's few
// entries per lane group, so its loads carry the streaming hint (ld_mat).  A
// tile with more than kSolTileCap entries is done as vector rows.  The trip
// count is uniform across the block.
constexpr int kSolTileLanes = 4;
constexpr int kSolTileRows = kBlock / kSolTileLanes;
constexpr int kSolTilePer = 4;
constexpr int kSolTileCap = kBlock * kSolTilePer;

// No epilogue operand: epi(row, total).  With a `pre` functor the epilogue is
// epi(row, total, pre(row)).  The vector form issues that load before the
// row's product, so that its latency overlaps the product's loads; the tile
// form loads it at the epilogue (its kernels use all 64 VGPRs, and an early
// load spilled: 241 -> 250 us per cabin iteration).
struct NoPre {
    __device__ int operator()(int64_t) const { return 0; }
};

template <typename T, typename Op, typename Epi, typename Pre = NoPre>
__device__ __forceinline__ void for_tiles(const Rows& rw, const int* __restrict__ rp, const int* __restrict__ ci,
                                          const cx<T>* __restrict__ vals, Op op, Epi epi, Pre pre = Pre{}) {
    constexpr bool kPre = !std::is_same_v<Pre, NoPre>;
    constexpr int L = kSolTileLanes;
    __shared__ cx<T> prod[kSolTileCap];
    const int t = threadIdx.x, g = t / L, lane = t % L;
    const int64_t first = rw.x0 + (int64_t)rw.k * kSolTileRows, step = (int64_t)rw.K * kSolTileRows;
    const int64_t r1 = rw.x1;
    for (int64_t r0 = first; r0 < r1; r0 += step) {
        const int64_t re = r0 + kSolTileRows < r1 ? r0 + kSolTileRows : r1;
        const int e0 = rp[r0], e1 = rp[re];
        const int64_t row = r0 + g;
        const int b = rp[row < re ? row : re], e = rp[row + 1 < re ? row + 1 : re];
        cx<T> acc = mk<T>(T(0), T(0));
        if (e1 > e0 && e1 - e0 <= kSolTileCap) {  // (a tile of empty rows loads nothing: block-uniform)
            const int last = e1 - 1;
            int c[kSolTilePer];
            cx<T> v[kSolTilePer], o[kSolTilePer];
#pragma unroll
            for (int k = 0; k < kSolTilePer; ++k) {
                const int p = e0 + t + k * kBlock;
                c[k] = ld_mat(ci + (p < last ? p : last));
            }
#pragma unroll
            for (int k = 0; k < kSolTilePer; ++k) {
                const int p = e0 + t + k * kBlock;
                v[k] = ld_mat(vals + (p < last ? p : last));
            }
#pragma unroll
            for (int k = 0; k < kSolTilePer; ++k) o[k] = op(c[k]);
#pragma unroll
            for (int k = 0; k < kSolTilePer; ++k) {
                const bool ok = e0 + t + k * kBlock < e1;
                const cx<T> pr = cmul<T>(v[k], o[k]);
                prod[t + k * kBlock] = mk<T>(ok ? pr.x : T(0), ok ? pr.y : T(0));
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
        if (row < re && lane == 0) {
            if constexpr (kPre) {
                epi(row, acc, pre(row));
            } else {
                epi(row, acc);
            }
        }
    }
}

// Row loop of a block over its tiles of RPS = kBlock/L rows (g = thread / L
// picks the row of the tile).  With
// PF the next step's row_ptr pair is loaded before the current row's product,
// so that load's latency overlaps the current step (two more live registers;
// kernels whose column functor gathers several vectors leave it off to stay
// within 64 VGPRs).  epi(row, total) runs in lane 0 of each row's group after
// the group sum.  The trip count is uniform across the block.
template <typename T, int L, int U, bool PF = true, typename Op, typename Epi, typename Pre = NoPre>
__device__ __forceinline__ void for_rows(const Rows& rw, const int* __restrict__ rp, const int* __restrict__ ci,
                                         const cx<T>* __restrict__ vals, Op op, Epi epi, Pre pre = Pre{}) {
    constexpr bool kPre = !std::is_same_v<Pre, NoPre>;
    if constexpr (L == 1) {
        for_tiles<T>(rw, rp, ci, vals, op, epi, pre);
        return;
    }
    constexpr int RPS = kBlock / L;
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    const int64_t first = rw.x0 + (int64_t)rw.k * RPS, step = (int64_t)rw.K * RPS, r1 = rw.x1;
    int64_t row = first + g;
    int beg = 0, end = 0;
    if (row < r1) {
        beg = rp[row];
        end = rp[row + 1];
    }
    for (int64_t base = first; base < r1; base += step) {
        const int64_t nrow = row + step;
        int nbeg = 0, nend = 0;
        if (PF && nrow < r1) {
            nbeg = rp[nrow];
            nend = rp[nrow + 1];
        }
        const bool ok = row < r1;
        if (!PF && ok && base != first) {
            beg = rp[row];
            end = rp[row + 1];
        }
        cx<T> acc = mk<T>(T(0), T(0));
        decltype(pre(row)) w{};
        if (ok) {
            if constexpr (kPre) w = pre(row);
            acc = row_partial<T, L, U>(beg, end, lane, ci, vals, op);
        }
        acc.x = group_sum<L>(acc.x);
        acc.y = group_sum<L>(acc.y);
        if (ok && lane == 0) {
            if constexpr (kPre) {
                epi(row, acc, w);
            } else {
                epi(row, acc);
            }
        }
        row = nrow;
        if (PF) {
            beg = nbeg;
            end = nend;
        }
    }
}

// ------------------------------------------------------------------ solver scalars (device resident)

// One block per system.  Written only by thread 0 of the system's first
// block, and read only by later kernels (never by other blocks of the
// writing kernel), except `done`, whose early read by other blocks of the
// system leads to the exit they would compute themselves.
struct alignas(256) SolverScal {
    double2 rho2[2];  // rho of iteration i in slot i & 1
    double2 alpha;    // alpha of the current iteration
    double2 omega;    // omega of the last completed iteration
    double2 beta;
    double bnorm;  // ||b||
    double rtol;
    double relres;       // last recursive ||r|| / ||b|| (or ||s|| / ||b||)
    double relres_true;  // filled by the final residual check
    double outer_rn;     // refinement: ||b - A x|| of the current outer step
    int iter;            // next iteration to run (1-based); written by the last kernel of an iteration
    int cur;             // iteration in progress; written by the first kernel of an iteration
    int maxiter;
    int status;  // solver status once done
    int done;    // 1 once the solve has ended (all later kernels are no-ops)
    int iters;   // reported iteration count
    int zero_x;  // ||b|| = 0: the solution is x = 0
    int bad_diag;  // Jacobi requested with a zero diagonal entry
    int pending;   // half-step exit taken in iteration `pending`; the next first kernel concludes
    int why;       // for a breakdown: which scalar vanished (BD_*)
};

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };
enum : int { BD_NONE = 0, BD_RHO = 1, BD_RHAT_V = 2, BD_TT = 3, BD_OMEGA = 4 };

// Reset the scalar blocks of nsys systems before a solve.
__global__ void k_sc_init(SolverScal* sc, int nsys, double rtol, int maxiter) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsys) return;
    SolverScal z = {};
    z.rtol = rtol;
    z.maxiter = maxiter;
    z.status = ST_NOT_CONVERGED;
    sc[j] = z;
}

// ------------------------------------------------------------------ work map of a solver launch

// Logical block lb of a solver launch belongs to system `sys`, takes the rows
// that (x0, x1, k, K) describe (as in struct Rows) of the (block-diagonal)
// matrix and is the `local`-th block of its system; sys < 0 marks padding.  System j owns the contiguous logical block
// range [gbeg, gbeg + gcnt).  A single solve is the one-system case.
struct BlockMap {
    int sys, x0, x1, k, K, local;  // rows as in struct Rows
};
struct SysMap {
    int gbeg, gcnt, row0, row1;
};

template <typename T> struct BicgArgs {
    int G;       // blocks of every solver launch (a multiple of 8, or < 8)
    int stride;  // partial component stride (>= pf G)
    int pf = 1;  // partial slots per block in regions A and B (sol_subs(G) when the products run as sub-blocks)
    const BlockMap* bmap;
    const SysMap* smap;
    int* ndone;  // systems finished so far
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const cx<T>* __restrict__ vals;
    const cx<T>* b;
    cx<T>* r;
    const cx<T>* rh;
    cx<T>* p[2];
    cx<T>* v[2];
    cx<T>* s;
    cx<T>* t;
    cx<T>* x;
    double* part;
    SolverScal* sc;
};

struct SysBlock {
    int lb, sys, local;
    Rows rw;
    int gbeg, gcnt;
};
template <typename T> __device__ __forceinline__ SysBlock sys_block(const BicgArgs<T>& a) {
    SysBlock q;
    q.lb = logical_block(blockIdx.x, a.G);
    const BlockMap m = a.bmap[q.lb];
    q.sys = m.sys;
    q.local = m.local;
    q.rw.x0 = m.x0;
    q.rw.x1 = m.x1;
    q.rw.k = m.k;
    q.rw.K = m.K;
    if (m.sys >= 0) {
        const SysMap sm = a.smap[m.sys];
        q.gbeg = sm.gbeg;
        q.gcnt = sm.gcnt;
    } else {
        q.gbeg = q.gcnt = 0;
    }
    return q;
}

__device__ __forceinline__ bool sys_leader(const SysBlock& q) { return q.local == 0 && threadIdx.x == 0; }

// Record the end of system q's solve (its leader thread only).
__device__ __forceinline__ void finish(SolverScal* sc, int* ndone, int status, int iterations, int why = BD_NONE) {
    sc->status = status;
    sc->iters = iterations;
    sc->why = why;
    sc->done = 1;
    atomicAdd(ndone, 1);
}

// Sum of K components over one system's partials [gbeg, gbeg + gcnt), in a
// fixed order, delivered to every thread of the block.
// Thread t takes partial t of every component; the K loads are issued
// together (so their latencies overlap).  Waves wholly past the partials
// load nothing (a wave-uniform branch); in the wave that straddles the end,
// the lanes past it read the last partial, a duplicate address that the
// load instruction merges (clamping every idle thread of every block to one
// address would make that address a hot spot).  A system's blocks never
// exceed kMaxGrid <= kBlock (gcnt >= 1); the loop for gcnt > kBlock only
// keeps the function general.
__device__ __forceinline__ int wave_base() {
    return __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~(kWave - 1);
}
template <int K>
__device__ __forceinline__ void sys_sum(const double* __restrict__ part, int stride, int gbeg, int gcnt,
                                        double (&out)[K]) {
    static_assert(kMaxGrid <= kBlock, "one partial per thread");
    __shared__ double bc[K];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    if (wave_base() < gcnt) {
        const bool mine = t < gcnt;
        const int g0 = gbeg + (mine ? t : gcnt - 1);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double v = part[k * stride + g0];
            out[k] = mine ? v : 0.0;
        }
    }
    if (gcnt > kBlock) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int g = t + kBlock; g < gcnt; g += kBlock) out[k] += part[k * stride + gbeg + g];
    }
    block_sum<K>(out);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) bc[k] = out[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = bc[k];
}

// Thread 0 writes the block's totals to slot pf lb of each component and
// zeros to the pf - 1 slots after it (a region whose other components come
// from a launch of pf times as many blocks).
template <int K>
__device__ __forceinline__ void store_sys_partials(double* __restrict__ part, int stride, int lb, double (&e)[K],
                                                   int pf = 1) {
    block_sum<K>(e);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            part[k * stride + pf * lb] = e[k];
            for (int f = 1; f < pf; ++f) part[k * stride + pf * lb + f] = 0.0;
        }
    }
}

// ------------------------------------------------------------------ standalone SpMV with residual epilogue

enum : int {
    EPI_NONE = 0,  // y = A x
    EPI_RESID = 1  // y = w - A x; partial ||y||^2 (1 component)
};

template <typename T> struct SpmvArgs {
    int n;
    Geom geo;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const cx<T>* __restrict__ vals;
    const cx<T>* __restrict__ x;
    cx<T>* __restrict__ y;
    const cx<T>* __restrict__ w;  // b for EPI_RESID
    double* __restrict__ part;    // region for EPI_RESID's partial
};

template <typename T, int L, int U, int EPI>
__global__ HZ_STREAM_BOUNDS void k_spmv(const SpmvArgs<T> a) {
    const RowRange rr = rows_of_block(a.n, a.geo);
    const cx<T>* __restrict__ xv = a.x;
    auto op = [xv](int c) { return xv[c]; };
    double e[1] = {0.0};
    for_rows<T, L, U>(rr.rw, a.row_ptr, a.col_idx, a.vals, op, [&](int64_t row, cx<T> acc) {
        if constexpr (EPI == EPI_RESID) {
            const cx<T> bw = a.w[row];
            acc.x = bw.x - acc.x;
            acc.y = bw.y - acc.y;
            e[0] = __builtin_fma((double)acc.x, (double)acc.x, e[0]);
            e[0] = __builtin_fma((double)acc.y, (double)acc.y, e[0]);
        }
        a.y[row] = acc;
    });
    if constexpr (EPI == EPI_RESID) store_partials<1>(a.part, rr.lb, e);
}

// y = b - A x over the solver's work map, per-system partial ||y||^2 in
// region I (the initial residual and the final true residual of a solve).
template <typename T, int L, int U>
__global__ HZ_STREAM_BOUNDS void k_sys_resid(const BicgArgs<T> a, const cx<T>* __restrict__ vals,
                                             const cx<T>* __restrict__ xin, cx<T>* __restrict__ y) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    auto op = [xin](int c) { return xin[c]; };
    double e[1] = {0.0};
    for_rows<T, L, U>(q.rw, a.row_ptr, a.col_idx, vals, op, [&](int64_t row, cx<T> acc) {
        const cx<T> bw = a.b[row];
        acc.x = bw.x - acc.x;
        acc.y = bw.y - acc.y;
        e[0] = __builtin_fma((double)acc.x, (double)acc.x, e[0]);
        e[0] = __builtin_fma((double)acc.y, (double)acc.y, e[0]);
        y[row] = acc;
    });
    store_sys_partials<1>(a.part + kPartI * a.stride, a.stride, q.lb, e);
}

// ------------------------------------------------------------------ BiCGStab: three kernels per iteration
//
// Iteration i (Section 7's P-BiCGSTAB, right-preconditioned; A here is the
// column-scaled matrix under Jacobi), for every system of the launch:
//   A-kernel: decide the end of iteration i-1 from <rhat,r>, ||r||; beta;
//             v = A p with p = r + beta (p_old - omega v_old) formed for every
//             gathered column; store p, v; partial <rhat, v>.
//   B-kernel: alpha = rho / <rhat, v>; t = A s with s = r - alpha v formed for
//             every gathered column; store s, t; partials ||s||^2, <t,s>, ||t||^2.
//   C-kernel: half-step test on ||s||; omega = <t,s>/<t,t>;
//             x += alpha p + omega s; r = s - omega t; partials <rhat,r>, ||r||^2.
// p and v are double-buffered by the parity of i, so the A-kernel reads the
// old vectors while writing the new ones.  Systems of a batch share nothing
// but the launches: each has its own scalars, partial range and exit.

// Start of iteration i = sc->iter for the block's system: conclude iteration
// i-1 (convergence on ||r||, breakdown, iteration limit) from the partials
// <rhat, r>, ||r||^2, then rho_i and beta.  Returns false when the system's
// solve has ended (every block of the system returns); its leader records
// the decision.
struct IterStart {
    int it;
    double2 rho, beta, omega;
};
// EARLY: the scalars written by earlier kernels are read before the
// reduction's barriers (a barrier is a fence, so loads after it cannot be
// hoisted above it), overlapping their latency with the partial loads; the
// fused A-kernel reads them after, as it has no registers to spare.
template <typename T, bool EARLY = true>
__device__ __forceinline__ bool iteration_start(const BicgArgs<T>& a, const SysBlock& q, IterStart& st) {
    if (q.sys < 0) return false;
    SolverScal* sc = a.sc + q.sys;
    if (sc->done) return false;
    if (sc->pending) {  // every block of the previous kernel has applied x += alpha p
        if (sys_leader(q)) finish(sc, a.ndone, ST_OK, sc->pending);
        return false;
    }
    const int it = sc->iter;
    double bnorm, rtol;
    int maxiter;
    double2 om_prev, rho_prev, al_prev;
    auto read = [&] {
        bnorm = sc->bnorm;
        rtol = sc->rtol;
        maxiter = sc->maxiter;
        om_prev = sc->omega;
        rho_prev = sc->rho2[(it - 1) & 1];
        al_prev = sc->alpha;
    };
    if constexpr (EARLY) read();
    double h[3];
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, q.gbeg, q.gcnt, h);
    if constexpr (!EARLY) read();
    const double2 rho = mk<double>(h[0], h[1]);
    double2 beta = mk<double>(0.0, 0.0), om = mk<double>(0.0, 0.0);
    if (it > 1) {
        const double rel = __builtin_sqrt(h[2]) / bnorm;
        om = om_prev;
        int stt = -1, sit = 0, why = BD_NONE;
        if (!__builtin_isfinite(rel)) stt = ST_NONFINITE, sit = it - 1;
        else if (rel <= rtol) stt = ST_OK, sit = it - 1;
        else if (zzero(om)) stt = ST_BREAKDOWN, sit = it - 1, why = BD_OMEGA;
        else if (it - 1 >= maxiter) stt = ST_NOT_CONVERGED, sit = maxiter;
        else if (!zfinite(rho)) stt = ST_NONFINITE, sit = it;
        else if (zzero(rho)) stt = ST_BREAKDOWN, sit = it, why = BD_RHO;
        else {
            beta = zmul(zdiv(rho, rho_prev), zdiv(al_prev, om));
            if (!zfinite(beta)) stt = ST_NONFINITE, sit = it;
        }
        if (sys_leader(q)) sc->relres = rel;
        if (stt >= 0) {
            if (sys_leader(q)) finish(sc, a.ndone, stt, sit, why);
            return false;
        }
    }
    if (sys_leader(q)) {
        sc->rho2[it & 1] = rho;
        sc->beta = beta;
        sc->cur = it;
    }
    st.it = it;
    st.rho = rho;
    st.beta = beta;
    st.omega = om;
    return true;
}

// p_i = r_i (first iteration) or r_i + beta (p_old_i - omega v_old_i)
template <typename T>
__device__ __forceinline__ cx<T> p_update(bool first, cx<T> bt, cx<T> omt, cx<T> rc, cx<T> pc, cx<T> vc) {
    if (first) return rc;
    const cx<T> d = mk<T>(pc.x - fmaT(omt.x, vc.x, -omt.y * vc.y), pc.y - fmaT(omt.x, vc.y, omt.y * vc.x));
    return cfma<T>(bt, d, rc);
}

template <typename T, int L, int U>
__global__ HZ_STREAM_BOUNDS void k_bicg_A(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    IterStart st;
    if (!iteration_start<T, false>(a, q, st)) return;
    const int it = st.it;
    const bool first = it == 1;
    const cx<T> bt = narrow<T>(st.beta), omt = narrow<T>(st.omega);
    const cx<T>* __restrict__ r = a.r;
    const cx<T>* __restrict__ pold = a.p[(it - 1) & 1];
    const cx<T>* __restrict__ vold = a.v[(it - 1) & 1];
    cx<T>* __restrict__ pnew = a.p[it & 1];
    cx<T>* __restrict__ vnew = a.v[it & 1];
    auto pcol = [=](int c) {
        if (first) return r[c];
        return p_update<T>(false, bt, omt, r[c], pold[c], vold[c]);
    };
    double e[2] = {0.0, 0.0};
    for_rows<T, L, U, false>(q.rw, a.row_ptr, a.col_idx, a.vals, pcol, [&](int64_t row, cx<T> acc) {
        pnew[row] = pcol((int)row);
        vnew[row] = acc;
        const cx<T> w = a.rh[row];
        double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
    });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

// alpha = rho / <rhat, v> for the block's system; false when the system ends here.
template <typename T>
__device__ __forceinline__ bool alpha_step(const BicgArgs<T>& a, const SysBlock& q, int& it, double2& alpha) {
    if (q.sys < 0) return false;
    SolverScal* sc = a.sc + q.sys;
    if (sc->done) return false;
    it = sc->cur;
    const double2 rho = sc->rho2[it & 1];  // written by the iteration's first kernel; read before the barriers
    double h[2];
    sys_sum<2>(a.part + kPartA * a.stride, a.stride, a.pf * q.gbeg, a.pf * q.gcnt, h);
    const double2 sigma = mk<double>(h[0], h[1]);
    if (!zfinite(sigma) || zzero(sigma)) {
        if (sys_leader(q)) finish(sc, a.ndone, zzero(sigma) ? ST_BREAKDOWN : ST_NONFINITE, it, zzero(sigma) ? BD_RHAT_V : BD_NONE);
        return false;
    }
    alpha = zdiv(rho, sigma);
    if (sys_leader(q)) sc->alpha = alpha;
    return true;
}

template <typename T, int L, int U>
__global__ HZ_STREAM_BOUNDS void k_bicg_B(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    int it;
    double2 alpha;
    if (!alpha_step(a, q, it, alpha)) return;
    const cx<T> al = narrow<T>(alpha);
    const cx<T>* __restrict__ r = a.r;
    const cx<T>* __restrict__ v = a.v[it & 1];
    auto scol = [=](int c) { return cfma<T>(mk<T>(-al.x, -al.y), v[c], r[c]); };
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for_rows<T, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, scol, [&](int64_t row, cx<T> acc) {
        const cx<T> s = scol((int)row);
        a.s[row] = s;
        a.t[row] = acc;
        e[0] = __builtin_fma((double)s.x, (double)s.x, e[0]);
        e[0] = __builtin_fma((double)s.y, (double)s.y, e[0]);
        double2 c = cdotacc(acc.x, acc.y, s.x, s.y, mk<double>(e[1], e[2]));
        e[1] = c.x;
        e[2] = c.y;
        e[3] = __builtin_fma((double)acc.x, (double)acc.x, e[3]);
        e[3] = __builtin_fma((double)acc.y, (double)acc.y, e[3]);
    });
    store_sys_partials<4>(a.part + kPartB * a.stride, a.stride, q.lb, e);
}

template <typename T>
__global__ HZ_STREAM_BOUNDS void k_bicg_C(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc + q.sys;
    if (sc->done) return;
    const int it = sc->cur;
    const double bnorm = sc->bnorm, rtol = sc->rtol;  // read before the reduction's barriers
    const double2 alpha = sc->alpha;
    double h[4];
    sys_sum<4>(a.part + kPartB * a.stride, a.stride, a.pf * q.gbeg, a.pf * q.gcnt, h);
    const double rel = __builtin_sqrt(h[0]) / bnorm;
    const cx<T> al = narrow<T>(alpha);
    const cx<T>* __restrict__ p = a.p[it & 1];
    if (!__builtin_isfinite(rel)) {
        if (sys_leader(q)) finish(sc, a.ndone, ST_NONFINITE, it);
        return;
    }
    if (rel <= rtol) {  // half-step exit: x += alpha p (concluded by the next first kernel)
        HZ_FOR_ELEMS(i, q.rw) a.x[i] = cfma<T>(al, p[i], a.x[i]);
        if (sys_leader(q)) {
            sc->relres = rel;
            sc->pending = it;
        }
        return;
    }
    const double2 ts = mk<double>(h[1], h[2]);
    const double tt = h[3];
    int st = -1, why = BD_NONE;
    double2 om = mk<double>(0.0, 0.0);
    if (!zfinite(ts) || !__builtin_isfinite(tt)) st = ST_NONFINITE;
    else if (tt == 0.0) st = ST_BREAKDOWN, why = BD_TT;
    else {
        om = zdiv(ts, mk<double>(tt, 0.0));
        if (!zfinite(om)) st = ST_NONFINITE;
    }
    if (st >= 0) {
        if (sys_leader(q)) finish(sc, a.ndone, st, it, why);
        return;
    }
    if (sys_leader(q)) {
        sc->omega = om;
        sc->iter = it + 1;
    }
    const cx<T> omt = narrow<T>(om), nom = mk<T>(-omt.x, -omt.y);
    double e[3] = {0.0, 0.0, 0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        const cx<T> sv = a.s[i], tv = a.t[i], rh = a.rh[i];
        cx<T> x = a.x[i];
        x = cfma<T>(al, p[i], x);
        x = cfma<T>(omt, sv, x);
        a.x[i] = x;
        const cx<T> r = cfma<T>(nom, tv, sv);
        a.r[i] = r;
        double2 c = cdotacc(rh.x, rh.y, r.x, r.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma((double)r.x, (double)r.x, e[2]);
        e[2] = __builtin_fma((double)r.y, (double)r.y, e[2]);
    }
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
}

// ------------------------------------------------------------------ gather-light variant (five kernels)
//
// For matrices whose column indices are far from the row (a random node
// numbering), forming p and s for every gathered column multiplies the
// number of scattered reads.  This variant materialises them first, so
// each product gathers one vector:
//   P-kernel: iteration_start, p = r + beta (p_old - omega v_old)   (element-wise)
//   A1-kernel: v = A p; partial <rhat, v>
//   S-kernel: alpha = rho / <rhat, v>; s = r - alpha v; partial ||s||^2
//   B1-kernel: t = A s; partials <t, s>, ||t||^2
//   C-kernel: as in the fused variant.

template <typename T>
__global__ HZ_STREAM_BOUNDS void k_bicg_P(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    IterStart st;
    if (!iteration_start(a, q, st)) return;
    const int it = st.it;
    const bool first = it == 1;
    const cx<T> bt = narrow<T>(st.beta), omt = narrow<T>(st.omega);
    const cx<T>* __restrict__ pold = a.p[(it - 1) & 1];
    const cx<T>* __restrict__ vold = a.v[(it - 1) & 1];
    cx<T>* __restrict__ pnew = a.p[it & 1];
    HZ_FOR_ELEMS(i, q.rw)
        pnew[i] = first ? a.r[i] : p_update<T>(false, bt, omt, a.r[i], pold[i], vold[i]);
}

template <typename T, int L, int U>
__global__ HZ_STREAM_BOUNDS void k_bicg_A1(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    const SolverScal* sc = a.sc + q.sys;
    if (sc->done || sc->pending) return;
    const int it = sc->cur;
    const cx<T>* __restrict__ p = a.p[it & 1];
    cx<T>* __restrict__ v = a.v[it & 1];
    auto pcol = [p](int c) { return p[c]; };
    const cx<T>* __restrict__ rh = a.rh;
    double e[2] = {0.0, 0.0};
    for_rows<T, L, U>(
        q.rw, a.row_ptr, a.col_idx, a.vals, pcol,
        [&](int64_t row, cx<T> acc, cx<T> w) {
            v[row] = acc;
            double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        },
        [rh](int64_t row) { return rh[row]; });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

template <typename T>
__global__ HZ_STREAM_BOUNDS void k_bicg_S(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    int it;
    double2 alpha;
    if (!alpha_step(a, q, it, alpha)) return;
    const cx<T> nal = mk<T>((T)-alpha.x, (T)-alpha.y);
    const cx<T>* __restrict__ v = a.v[it & 1];
    double e[1] = {0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        const cx<T> s = cfma<T>(nal, v[i], a.r[i]);
        a.s[i] = s;
        e[0] = __builtin_fma((double)s.x, (double)s.x, e[0]);
        e[0] = __builtin_fma((double)s.y, (double)s.y, e[0]);
    }
    store_sys_partials<1>(a.part + kPartB * a.stride, a.stride, q.lb, e, a.pf);
}

template <typename T, int L, int U>
__global__ HZ_STREAM_BOUNDS void k_bicg_B1(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    if (a.sc[q.sys].done) return;
    const cx<T>* __restrict__ sv = a.s;
    auto scol = [sv](int c) { return sv[c]; };
    double e[3] = {0.0, 0.0, 0.0};
    for_rows<T, L, U>(
        q.rw, a.row_ptr, a.col_idx, a.vals, scol,
        [&](int64_t row, cx<T> acc, cx<T> s) {
            a.t[row] = acc;
            double2 c = cdotacc(acc.x, acc.y, s.x, s.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
            e[2] = __builtin_fma((double)acc.x, (double)acc.x, e[2]);
            e[2] = __builtin_fma((double)acc.y, (double)acc.y, e[2]);
        },
        [sv](int64_t row) { return sv[row]; });
    store_sys_partials<3>(a.part + (kPartB + 1) * a.stride, a.stride, q.lb, e);
}

// Locality of a CSR matrix: count of entries with |col - row| > W (integer atomics).
__global__ __launch_bounds__(kBlock) void k_far_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                      int W, unsigned long long* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double c = 0.0;  // exact: counts stay far below 2^53
    if (i < n)
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t d = (int64_t)ci[p] - i;
            c += (d > W || d < -W) ? 1.0 : 0.0;
        }
    c = group_sum<64>(c);
    if (threadIdx.x % kWave == 0 && c != 0.0) atomicAdd(count, (unsigned long long)c);
}

// Solve set-up: r = src (b, or the residual b - A x0), rhat = r;
// partials <rhat, r>, ||r||^2 (region C) and ||b||^2 (region I).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const BicgArgs<T> a, const cx<T>* src) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    double e[3] = {0.0, 0.0, 0.0}, eb[1] = {0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        const cx<T> bv = a.b[i], rv = src[i];
        if (a.r != src) a.r[i] = rv;
        const_cast<cx<T>*>(a.rh)[i] = rv;
        eb[0] = __builtin_fma((double)bv.x, (double)bv.x, eb[0]);
        eb[0] = __builtin_fma((double)bv.y, (double)bv.y, eb[0]);
        double2 c = cdotacc(rv.x, rv.y, rv.x, rv.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma((double)rv.x, (double)rv.x, e[2]);
        e[2] = __builtin_fma((double)rv.y, (double)rv.y, e[2]);
    }
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
    store_sys_partials<1>(a.part + kPartI * a.stride, a.stride, q.lb, eb);
}

// ||b||, initial convergence test, per system (one block per system); iteration 1 comes next.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_init(const BicgArgs<T> a) {
    const int j = blockIdx.x;
    const SysMap sm = a.smap[j];
    SolverScal* sc = a.sc + j;
    double hb[1], hr[3];
    sys_sum<1>(a.part + kPartI * a.stride, a.stride, sm.gbeg, sm.gcnt, hb);
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, sm.gbeg, sm.gcnt, hr);
    if (threadIdx.x != 0) return;
    const double bn = __builtin_sqrt(hb[0]);
    sc->bnorm = bn;
    sc->iter = 1;
    sc->cur = 0;
    sc->done = 0;
    sc->zero_x = 0;
    sc->iters = 0;
    sc->pending = 0;
    sc->why = BD_NONE;
    sc->status = ST_NOT_CONVERGED;
    sc->alpha = sc->omega = sc->beta = mk<double>(1.0, 0.0);
    if (!__builtin_isfinite(bn) || !__builtin_isfinite(hr[2])) return finish(sc, a.ndone, ST_NONFINITE, 0);
    if (bn == 0.0) {
        sc->zero_x = 1;
        sc->relres = 0.0;
        return finish(sc, a.ndone, ST_OK, 0);
    }
    const double rel = __builtin_sqrt(hr[2]) / bn;
    sc->relres = rel;
    if (rel <= sc->rtol) finish(sc, a.ndone, ST_OK, 0);
    else if (sc->maxiter <= 0) finish(sc, a.ndone, ST_NOT_CONVERGED, 0);
}

// relres_true = sqrt(region I over the system) / ||b||, one block per system
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_true(const BicgArgs<T> a) {
    const int j = blockIdx.x;
    const SysMap sm = a.smap[j];
    double h[1];
    sys_sum<1>(a.part + kPartI * a.stride, a.stride, sm.gbeg, sm.gcnt, h);
    SolverScal* sc = a.sc + j;
    if (threadIdx.x == 0) sc->relres_true = sc->bnorm > 0.0 ? __builtin_sqrt(h[0]) / sc->bnorm : 0.0;
}

// x = 0 on the rows of systems whose right-hand side is zero
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_if(const BicgArgs<T> a) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0 || !a.sc[q.sys].zero_x) return;
    HZ_FOR_ELEMS(i, q.rw) a.x[i] = mk<T>(T(0), T(0));
}

// ------------------------------------------------------------------ Jacobi folding: A D^{-1}

// dinv_i = 1 / A_ii ; flags a missing or zero diagonal.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const cx<T>* __restrict__ vals, cx<T>* __restrict__ dinv,
                                                        SolverScal* sc) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    cx<T> d = mk<T>(T(0), T(0));
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = vals[p];
    if (d.x == T(0) && d.y == T(0)) {
        sc->bad_diag = 1;  // every writer stores 1
        dinv[i] = mk<T>(T(0), T(0));
        return;
    }
    const T q = d.x * d.x + d.y * d.y;
    dinv[i] = mk<T>(d.x / q, -d.y / q);
}

// scaled_p = vals_p * dinv[col_p]   (column scaling A D^{-1})
template <typename T>
__global__ __launch_bounds__(kBlock) void k_colscale(int64_t nnz, const int* __restrict__ ci, const cx<T>* __restrict__ vals,
                                                     const cx<T>* __restrict__ dinv, cx<T>* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nnz) return;
    out[p] = cmul<T>(vals[p], dinv[ci[p]]);
}

// y_i = d_i x_i with d = 1 / dinv (the preconditioned initial iterate), or x_i = dinv_i y_i at the end
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_apply(int n, const cx<T>* __restrict__ dinv, cx<T>* __restrict__ x,
                                                       int invert) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    cx<T> d = dinv[i];
    if (invert) {
        const T q = d.x * d.x + d.y * d.y;
        d = mk<T>(d.x / q, -d.y / q);
    }
    x[i] = cmul<T>(d, x[i]);
}


// ------------------------------------------------------------------ standalone BLAS-1

template <int MODE>  // 0: conj(x) y  (2 comps), 1: |x|^2 (1 comp)
__global__ __launch_bounds__(kBlock) void k_dot_part(int n, Geom geo, const double2* __restrict__ x,
                                                     const double2* __restrict__ y, double* __restrict__ part) {
    const RowRange rr = rows_of_block(n, geo);
    constexpr int K = MODE == 0 ? 2 : 1;
    double e[K];
#pragma unroll
    for (int k = 0; k < K; ++k) e[k] = 0.0;
    HZ_FOR_ELEMS(i, rr.rw) {
        const double2 xv = x[i];
        if constexpr (MODE == 0) {
            const double2 yv = y[i];
            double2 c = cdotacc(xv.x, xv.y, yv.x, yv.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        } else {
            e[0] = __builtin_fma(xv.x, xv.x, e[0]);
            e[0] = __builtin_fma(xv.y, xv.y, e[0]);
        }
    }
    store_partials<K>(part, rr.lb, e);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_dot_fin(const double* __restrict__ part, int G, void* out) {
    constexpr int K = MODE == 0 ? 2 : 1;
    double s[K];
    head_sum<K>(part, G, s);
    if (threadIdx.x != 0) return;
    if constexpr (MODE == 0) {
        static_cast<double2*>(out)[0] = mk<double>(s[0], s[1]);
    } else {
        static_cast<double*>(out)[0] = __builtin_sqrt(s[0]);
    }
}

__global__ __launch_bounds__(kBlock) void k_zaxpy(int64_t n, double2 alpha, const double2* __restrict__ x,
                                                  double2* __restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) y[i] = cfma<double>(alpha, x[i], y[i]);
}

// ------------------------------------------------------------------ CSR validation

__global__ __launch_bounds__(kBlock) void k_validate(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > n) return;
    const int a = rp[i];
    if (i == 0 && a != 0) *bad = 1;
    if (i == n) {
        if (a != nnz) *bad = 1;
        return;
    }
    const int b = rp[i + 1];
    if (b < a || a < 0 || b > nnz) {
        *bad = 1;
        return;
    }
    for (int p = a; p < b; ++p)
        if (ci[p] < 0 || ci[p] >= n) {
            *bad = 1;
            return;
        }
}

}  // namespace hz

// ================================================================== mixed precision (complex64 inner solve)
namespace hz {

// out32_p = complex64(vals_p * dinv[col_p]) (Jacobi) or complex64(vals_p)
__global__ __launch_bounds__(kBlock) void k_demote_vals(int64_t nnz, const int* __restrict__ ci,
                                                        const double2* __restrict__ vals,
                                                        const double2* __restrict__ dinv, float2* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nnz) return;
    double2 v = vals[p];
    if (dinv != nullptr) v = cmul<double>(v, dinv[ci[p]]);
    out[p] = mk<float>((float)v.x, (float)v.y);
}

__global__ __launch_bounds__(kBlock) void k_demote_vec(int n, const double2* __restrict__ in, float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double2 v = in[i];
    out[i] = mk<float>((float)v.x, (float)v.y);
}

// Outer scalars of the refinement live in a second SolverScal: bnorm, relres,
// status/done, and outer_rn = ||r|| of the current outer residual.
__global__ __launch_bounds__(kBlock) void k_fin_bnorm(const double* __restrict__ part, int G, SolverScal* sc) {
    double s[1];
    head_sum<1>(part, G, s);
    if (threadIdx.x == 0) sc->bnorm = __builtin_sqrt(s[0]);
}

// After r = b - A x: decide convergence; otherwise record ||r|| for the next correction.
__global__ __launch_bounds__(kBlock) void k_fin_outer(const double* __restrict__ part, int G, SolverScal* sc,
                                                      int outer, int max_outer) {
    double s[1];
    head_sum<1>(part, G, s);
    if (threadIdx.x != 0) return;
    const double rn = __builtin_sqrt(s[0]), bn = sc->bnorm;
    sc->outer_rn = rn;
    int st = -1;
    if (!__builtin_isfinite(rn) || !__builtin_isfinite(bn)) st = ST_NONFINITE;
    else if (bn == 0.0) {
        sc->zero_x = 1;
        sc->relres = 0.0;
        st = ST_OK;
    } else {
        const double rel = rn / bn;
        sc->relres = rel;
        sc->relres_true = rel;
        if (rel <= sc->rtol) st = ST_OK;
        else if (outer >= max_outer) st = ST_NOT_CONVERGED;
    }
    if (st >= 0) {
        sc->status = st;
        sc->iters = outer;
        sc->done = 1;
    }
}

// b32 = complex64(r / ||r||)
__global__ __launch_bounds__(kBlock) void k_demote_scaled(int n, const double2* __restrict__ r, const SolverScal* sc,
                                                          float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / sc->outer_rn;
    const double2 v = r[i];
    out[i] = mk<float>((float)(v.x * inv), (float)(v.y * inv));
}

// x += ||r|| * D^{-1} d  (FP64 update of the FP64 iterate)
__global__ __launch_bounds__(kBlock) void k_promote_add(int n, const float2* __restrict__ d, const float2* __restrict__ dinv,
                                                        const SolverScal* sc, double2* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double rn = sc->outer_rn;
    double2 dv = mk<double>((double)d[i].x, (double)d[i].y);
    if (dinv != nullptr) dv = zmul(mk<double>((double)dinv[i].x, (double)dinv[i].y), dv);
    double2 xv = x[i];
    xv.x = __builtin_fma(rn, dv.x, xv.x);
    xv.y = __builtin_fma(rn, dv.y, xv.y);
    x[i] = xv;
}

}  // namespace hz
