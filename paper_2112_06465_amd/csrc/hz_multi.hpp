// Shared-pattern batched BiCGStab: B systems A_j x_j = b_j with one sparsity
// pattern, e.g. a frequency sweep A(k_j) = K - k_j^2 M + i k_j B on one mesh.
// Each system runs Section 7's preconditioned BiCGStab with its own scalars,
// convergence test and exit; the systems share the launches, the row_ptr /
// col_idx reads and the gathers' cache lines.
//
// Layout (system-minor): entry p of system j is vals[p*B + j]; element i of
// a vector of system j is v[i*B + j].  A block owns a contiguous row chunk
// (XCD-aware mapping as in the single solve) and takes kBlock/BL rows per
// step with one lane per system (BL = a power of two >= B; lanes j >= B
// idle).  A row's values and gathered x of all systems are then contiguous
// B*16-byte runs: every load is coalesced, col_idx is read once for all
// systems, and no cross-lane row reduction is needed.
//
// Iteration (gather-light, five kernels, as for randomly numbered single
// systems):
//   P:  conclude iteration i-1 per system (<rhat,r>, ||r||), beta;
//       p = r + beta (p - omega v)
//   A1: v = A p; partial <rhat, v>
//   S:  alpha = rho / <rhat, v>; s = r - alpha v; partial ||s||^2
//   B1: t = A s; partials <t, s>, ||t||^2
//   C:  half-step test; omega = <t,s>/<t,t>; x += alpha p + omega s;
//       r = s - omega t; partials <rhat, r>, ||r||^2
// Partials are per (component, block, lane), reduced over the row slots of a
// block by a fixed tree and finished at the consumer's head by every block
// in a fixed order: reruns are bitwise identical, and system j's arithmetic
// does not depend on the other systems (permuting the batch permutes the
// results bitwise).
#pragma once

#include "hz_kernels.hpp"

namespace hz {

constexpr int kMultiMax = 256;  // most systems per shared-pattern launch

// Where the row product takes system j's entry p from.
enum : int {
    VS_EXPLICIT = 0,  // vals[p*B + j] (column-scaled by D_j^{-1} under Jacobi)
    VS_KMB = 1        // K[p] - k_j^2 M[p] + i k_j Bm[p] (a frequency sweep; never scaled)
};

struct MultiArgs {
    int n;     // rows of the shared pattern
    int B;     // systems
    Geom geo;  // row chunks of the geo.G blocks
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const double2* __restrict__ vals;  // VS_EXPLICIT: [nnz][B]
    const double* __restrict__ K;      // VS_KMB: three real [nnz] arrays and the wavenumbers [B]
    const double* __restrict__ M;
    const double* __restrict__ Bm;
    const double* __restrict__ kw;
    const double2* dinv;  // non-null: the products act on q = D^{-1} p and u = D^{-1} s ([n][B])
    const double* kd;     // VS_KMB with Jacobi, instead of dinv: row i's diagonal K, M, Bm at kd[4 i .. 4 i + 2]
    const double2* b;     // [n][B]
    double2* r;
    double2* rh;
    double2* p;
    double2* v;
    double2* s;
    double2* t;
    double2* q;  // the vector A1 gathers: p itself, or D^{-1} p written by P
    double2* u;  // the vector B1 gathers: s itself, or D^{-1} s written by S
    double2* x;
    double* part;    // [kParts][G][BL]
    SolverScal* sc;  // [B]
    int* ndone;      // systems finished so far
};

// Sum v[k] over the row slots of the block separately for every lane, by a
// fixed tree over slots; every thread receives the sums of its lane.
template <int BL, int K>
__device__ __forceinline__ void slot_sum(double (&v)[K]) {
    constexpr int S = kBlock / BL;
    __shared__ double red[K][kBlock];
    const int t = threadIdx.x;
    __syncthreads();  // a previous use of red has been read
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][t] = v[k];
    __syncthreads();
#pragma unroll
    for (int s = S / 2; s >= 1; s /= 2) {
        if (t < s * BL) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[k][t] += red[k][t + s * BL];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[k][t % BL];
}

// The block's partials of K components: region[(k*G + lb)*BL + lane].
template <int BL, int K>
__device__ __forceinline__ void mstore(double* region, int G, int lb, double (&e)[K]) {
    slot_sum<BL, K>(e);
    if (threadIdx.x < BL) {
#pragma unroll
        for (int k = 0; k < K; ++k) region[((size_t)k * G + lb) * BL + threadIdx.x] = e[k];
    }
}

// Totals of K components over all G blocks for the thread's lane.
template <int BL, int K>
__device__ __forceinline__ void mhead(const double* region, int G, double (&out)[K]) {
    constexpr int S = kBlock / BL;
    const int g = threadIdx.x / BL, j = threadIdx.x % BL;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int b = g; b < G; b += S) s += region[((size_t)k * G + b) * BL + j];
        out[k] = s;
    }
    slot_sum<BL, K>(out);
}

// True when every system has ended.  One read per block, broadcast through
// LDS, so all waves of the block take the same branch (the counter may grow
// while the kernel runs: leaders of P, S and C finish systems).
__device__ __forceinline__ bool all_done(const MultiArgs& a) {
    __shared__ int flag;
    if (threadIdx.x == 0) flag = *a.ndone >= a.B;
    __syncthreads();
    return flag != 0;
}

template <int BL> __device__ __forceinline__ double* mregion(const MultiArgs& a, int comp) {
    return a.part + (size_t)comp * a.geo.G * BL;
}

// The leader of system j: lane j of row slot 0 in logical block 0.
template <int BL> __device__ __forceinline__ bool mleader(int lb) { return lb == 0 && threadIdx.x < BL; }

// Entry p of system j.  k = (k_j, k_j^2) for VS_KMB.
template <int VS>
__device__ __forceinline__ double2 mval(const MultiArgs& a, int p, int j, double2 k) {
    if constexpr (VS == VS_EXPLICIT) {
        return a.vals[(size_t)p * a.B + j];
    } else {
        return mk<double>(__builtin_fma(-k.y, a.M[p], a.K[p]), k.x * a.Bm[p]);
    }
}

template <int VS> __device__ __forceinline__ double2 mwave(const MultiArgs& a, int j) {
    if constexpr (VS == VS_KMB) {
        const double kj = a.kw[j];
        return mk<double>(kj, kj * kj);
    } else {
        return mk<double>(0.0, 0.0);
    }
}

// Row i of A times X for lane j: entries in order, U loads of each kind in flight.
template <int U, int VS>
__device__ __forceinline__ double2 mrow(const MultiArgs& a, int64_t i, int j, const double2* __restrict__ X,
                                        double2 k) {
    const size_t B = (size_t)a.B;
    const int beg = a.row_ptr[i], end = a.row_ptr[i + 1];
    double2 acc = mk<double>(0.0, 0.0);
    int p = beg;
    for (; p + U <= end; p += U) {
        int c[U];
        double2 av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = a.col_idx[p + u];
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = mval<VS>(a, p + u, j, k);
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[(size_t)c[u] * B + j];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = cfma<double>(av[u], xv[u], acc);
    }
    for (; p < end; ++p) acc = cfma<double>(mval<VS>(a, p, j, k), X[(size_t)a.col_idx[p] * B + j], acc);
    return acc;
}

// The products stage a tile's column indices (and, for K/M/B, its K, M, Bm
// entries) in LDS: every lane of a row (one per system) needs the same ones,
// and loading them per lane costs one 64-lane load instruction per entry and
// kind for BL times fewer distinct values.  Explicit values differ per system
// and are still loaded per lane.  Tiles with more entries than kMTileCap read
// everything per lane as mrow does.
constexpr int kMTileCap = 1536;

// Row i of A_j times X for lane j, entries [b, e) of the staged tile (tile
// offsets; the tile starts at entry e0); the same operations in the same
// order as mrow<U, VS>, so the results are bitwise equal.
template <int U, int VS>
__device__ __forceinline__ double2 mrow_lds(const MultiArgs& a, int e0, const int* cs, const double* ks,
                                            const double* ms, const double* bs, int b, int e, int j, size_t B,
                                            const double2* __restrict__ X, double2 k) {
    auto val = [&](int p) {
        if constexpr (VS == VS_KMB) {
            return mk<double>(__builtin_fma(-k.y, ms[p], ks[p]), k.x * bs[p]);
        } else {
            return ld_mat(a.vals + (size_t)(e0 + p) * B + j);
        }
    };
    double2 acc = mk<double>(0.0, 0.0);
    int p = b;
    for (; p + U <= e; p += U) {
        int c[U];
        double2 xv[U], av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cs[p + u];
        if constexpr (VS != VS_KMB) {
#pragma unroll
            for (int u = 0; u < U; ++u) av[u] = val(p + u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[(size_t)c[u] * B + j];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = cfma<double>(VS == VS_KMB ? val(p + u) : av[u], xv[u], acc);
    }
    for (; p < e; ++p) acc = cfma<double>(val(p), X[(size_t)cs[p] * B + j], acc);
    return acc;
}

// f(i, acc, w) for every row i of the block on lane j when `on`, acc = row i
// of A_j times X and w = pre(i), an operand of the epilogue.  The block walks
// its rows in tiles of kBlock / BL consecutive rows (the rows and order of
// HZ_MROWS); a tile's shared entries are loaded once, contiguously by the
// whole block, into LDS.  The row's bounds are loaded with the tile's (before
// the staging) and w before the row's gathers, so neither load adds a wait
// of its own after the barrier.
template <int BL, int U, int VS, typename P, typename F>
__device__ __forceinline__ void m_tiles(const MultiArgs& a, const RowRange& rr, bool on, const double2* __restrict__ X,
                                        double2 k, P&& pre, F&& f) {
    constexpr int S = kBlock / BL;
    constexpr bool kmb = VS == VS_KMB;
    constexpr int KC = kmb ? kMTileCap : 1;  // K, M, Bm staged only for K/M/B
    __shared__ int cs[kMTileCap];
    __shared__ double ks[KC], ms[KC], bs[KC];
    const int g = threadIdx.x / BL, j = threadIdx.x % BL;
    const int* __restrict__ rp = a.row_ptr;
    for (int64_t r0 = rr.rw.x0 + (int64_t)rr.rw.k * S; r0 < rr.rw.x1; r0 += (int64_t)rr.rw.K * S) {  // uniform
        const int64_t re = r0 + S < rr.rw.x1 ? r0 + S : rr.rw.x1;
        const int64_t i = r0 + g, ic = i < re ? i : re - 1;  // ic: an in-bounds row of the tile
        const int e0 = rp[r0], ne = rp[re] - e0;
        const int rb = rp[ic], rend = rp[ic + 1];
        const bool staged = ne <= kMTileCap;
        if (staged) {
            for (int q = threadIdx.x; q < ne; q += kBlock) {
                cs[q] = a.col_idx[e0 + q];
                if constexpr (kmb) {
                    ks[q] = a.K[e0 + q];
                    ms[q] = a.M[e0 + q];
                    bs[q] = a.Bm[e0 + q];
                }
            }
            __syncthreads();
        }
        if (on && i < re) {
            const double2 w = pre(i);
            const double2 acc = staged ? mrow_lds<(kmb || U < 3 ? U : 3), VS>(a, e0, cs, ks, ms, bs, rb - e0, rend - e0, j, (size_t)a.B, X, k)
                                       : mrow<2, VS>(a, i, j, X, k);
            f(i, acc, w);
        }
        if (staged) __syncthreads();  // the tile's entries have been read
    }
}

// 1 / (K_ii - k^2 M_ii + i k Bm_ii) from the row's diagonal triple, with the
// operations of k_m_jacobi_kmb (bitwise the value it stores in dinv).
__device__ __forceinline__ double2 m_dinv_kmb(const double* __restrict__ kd, int64_t i, double kj) {
    const double2 km = reinterpret_cast<const double2*>(kd)[2 * i];
    const double bd = kd[4 * i + 2];
    const double2 d = mk<double>(__builtin_fma(-kj * kj, km.y, km.x), kj * bd);
    const double q = d.x * d.x + d.y * d.y;
    return mk<double>(d.x / q, -d.y / q);
}

#define HZ_MULTI_ROWS                                       \
    constexpr int S = kBlock / BL;                          \
    const RowRange rr = rows_of_block(a.n, a.geo);          \
    const int g = threadIdx.x / BL, j = threadIdx.x % BL;   \
    const size_t Bz = (size_t)a.B;                          \
    (void)Bz

// The block's rows for slot g: its tiles of S rows (see struct Rows).
#define HZ_MROWS(i) \
    for (int64_t i = rr.rw.x0 + (int64_t)rr.rw.k * S + g; i < rr.rw.x1; i += (int64_t)rr.rw.K * S)

// Solve set-up: r = src, rhat = src; partials <rhat,r>, ||r||^2 (C), ||b||^2 (I).
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_init(const MultiArgs a, const double2* src) {
    HZ_MULTI_ROWS;
    double e[3] = {0.0, 0.0, 0.0}, eb[1] = {0.0};
    if (j < a.B)
        HZ_MROWS(i) {
            const size_t q = (size_t)i * Bz + j;
            const double2 bv = a.b[q], rv = src[q];
            if (a.r != src) a.r[q] = rv;
            a.rh[q] = rv;
            eb[0] = __builtin_fma(bv.x, bv.x, eb[0]);
            eb[0] = __builtin_fma(bv.y, bv.y, eb[0]);
            const double2 c = cdotacc(rv.x, rv.y, rv.x, rv.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
            e[2] = __builtin_fma(rv.x, rv.x, e[2]);
            e[2] = __builtin_fma(rv.y, rv.y, e[2]);
        }
    mstore<BL, 3>(mregion<BL>(a, kPartC), a.geo.G, rr.lb, e);
    mstore<BL, 1>(mregion<BL>(a, kPartI), a.geo.G, rr.lb, eb);
}

// ||b||, initial convergence test of every system (one block).
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_fin_init(const MultiArgs a) {
    double hb[1], hr[3];
    mhead<BL, 1>(mregion<BL>(a, kPartI), a.geo.G, hb);
    mhead<BL, 3>(mregion<BL>(a, kPartC), a.geo.G, hr);
    const int j = threadIdx.x;
    if (j >= a.B) return;  // lanes of slot 0 only (B <= BL)
    SolverScal* sc = a.sc + j;
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

// P-kernel: end of iteration i-1 and beta per system (as in the single
// solve), then p = r + beta (p - omega v) on the system's lanes.
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_P(const MultiArgs a) {
    if (all_done(a)) return;
    HZ_MULTI_ROWS;
    double h[3];
    mhead<BL, 3>(mregion<BL>(a, kPartC), a.geo.G, h);
    if (j >= a.B) return;
    SolverScal* sc = a.sc + j;
    const bool lead = mleader<BL>(rr.lb);
    if (sc->done) return;
    if (sc->pending) {  // the half step's x += alpha p is complete everywhere
        if (lead) finish(sc, a.ndone, ST_OK, sc->pending);
        return;
    }
    const int it = sc->iter;
    const double2 rho = mk<double>(h[0], h[1]);
    double2 beta = mk<double>(0.0, 0.0), om = mk<double>(0.0, 0.0);
    if (it > 1) {
        const double rel = __builtin_sqrt(h[2]) / sc->bnorm;
        om = sc->omega;
        int stt = -1, sit = 0, why = BD_NONE;
        if (!__builtin_isfinite(rel)) stt = ST_NONFINITE, sit = it - 1;
        else if (rel <= sc->rtol) stt = ST_OK, sit = it - 1;
        else if (zzero(om)) stt = ST_BREAKDOWN, sit = it - 1, why = BD_OMEGA;
        else if (it - 1 >= sc->maxiter) stt = ST_NOT_CONVERGED, sit = sc->maxiter;
        else if (!zfinite(rho)) stt = ST_NONFINITE, sit = it;
        else if (zzero(rho)) stt = ST_BREAKDOWN, sit = it, why = BD_RHO;
        else {
            beta = zmul(zdiv(rho, sc->rho2[(it - 1) & 1]), zdiv(sc->alpha, om));
            if (!zfinite(beta)) stt = ST_NONFINITE, sit = it;
        }
        if (lead) sc->relres = rel;
        if (stt >= 0) {
            if (lead) finish(sc, a.ndone, stt, sit, why);
            return;
        }
    }
    if (lead) {
        sc->rho2[it & 1] = rho;
        sc->beta = beta;
        sc->cur = it;
    }
    const double kj = a.kd ? a.kw[j] : 0.0;
    HZ_MROWS(i) {
        const size_t q = (size_t)i * Bz + j;
        const double2 rv = a.r[q];
        double2 pn = rv;
        if (it != 1) {
            const double2 pv = a.p[q], vv = a.v[q];
            const double2 d = mk<double>(pv.x - __builtin_fma(om.x, vv.x, -om.y * vv.y),
                                         pv.y - __builtin_fma(om.x, vv.y, om.y * vv.x));
            pn = cfma<double>(beta, d, rv);
        }
        a.p[q] = pn;
        if (a.kd) a.q[q] = cmul<double>(m_dinv_kmb(a.kd, i, kj), pn);
        else if (a.dinv) a.q[q] = cmul<double>(a.dinv[q], pn);
    }
}

// A1-kernel: v = A p; partial <rhat, v>.
template <int BL, int U, int VS>
__global__ HZ_STREAM_BOUNDS void k_m_A1(const MultiArgs a) {
    if (all_done(a)) return;
    HZ_MULTI_ROWS;
    double e[2] = {0.0, 0.0};
    const bool on = j < a.B && !a.sc[j].done && !a.sc[j].pending;
    auto pre = [&](int64_t i) { return a.rh[(size_t)i * Bz + j]; };
    auto row = [&](int64_t i, double2 acc, double2 w) {
        a.v[(size_t)i * Bz + j] = acc;
        const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
    };
    m_tiles<BL, U, VS>(a, rr, on, a.q, j < a.B ? mwave<VS>(a, j) : mk<double>(0.0, 0.0), pre, row);
    mstore<BL, 2>(mregion<BL>(a, kPartA), a.geo.G, rr.lb, e);
}

// S-kernel: alpha = rho / <rhat, v>; s = r - alpha v; partial ||s||^2.
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_S(const MultiArgs a) {
    if (all_done(a)) return;
    HZ_MULTI_ROWS;
    double h[2], e[1] = {0.0};
    mhead<BL, 2>(mregion<BL>(a, kPartA), a.geo.G, h);
    bool go = j < a.B;
    double2 alpha = mk<double>(0.0, 0.0);
    if (go) {
        SolverScal* sc = a.sc + j;
        go = !sc->done && !sc->pending;
        if (go) {
            const int it = sc->cur;
            const double2 sigma = mk<double>(h[0], h[1]);
            if (!zfinite(sigma) || zzero(sigma)) {
                if (mleader<BL>(rr.lb)) finish(sc, a.ndone, zzero(sigma) ? ST_BREAKDOWN : ST_NONFINITE, it, zzero(sigma) ? BD_RHAT_V : BD_NONE);
                go = false;
            } else {
                alpha = zdiv(sc->rho2[it & 1], sigma);
                if (mleader<BL>(rr.lb)) sc->alpha = alpha;
            }
        }
    }
    if (go) {
        const double2 nal = mk<double>(-alpha.x, -alpha.y);
        const double kj = a.kd ? a.kw[j] : 0.0;
        HZ_MROWS(i) {
            const size_t q = (size_t)i * Bz + j;
            const double2 sv = cfma<double>(nal, a.v[q], a.r[q]);
            a.s[q] = sv;
            if (a.kd) a.u[q] = cmul<double>(m_dinv_kmb(a.kd, i, kj), sv);
            else if (a.dinv) a.u[q] = cmul<double>(a.dinv[q], sv);
            e[0] = __builtin_fma(sv.x, sv.x, e[0]);
            e[0] = __builtin_fma(sv.y, sv.y, e[0]);
        }
    }
    mstore<BL, 1>(mregion<BL>(a, kPartB), a.geo.G, rr.lb, e);
}

// B1-kernel: t = A s; partials <t, s>, ||t||^2.
template <int BL, int U, int VS>
__global__ HZ_STREAM_BOUNDS void k_m_B1(const MultiArgs a) {
    if (all_done(a)) return;
    HZ_MULTI_ROWS;
    double e[3] = {0.0, 0.0, 0.0};
    const bool on = j < a.B && !a.sc[j].done;
    auto pre = [&](int64_t i) { return a.s[(size_t)i * Bz + j]; };
    auto row = [&](int64_t i, double2 acc, double2 sv) {
        a.t[(size_t)i * Bz + j] = acc;
        const double2 c = cdotacc(acc.x, acc.y, sv.x, sv.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma(acc.x, acc.x, e[2]);
        e[2] = __builtin_fma(acc.y, acc.y, e[2]);
    };
    m_tiles<BL, U, VS>(a, rr, on, a.u, j < a.B ? mwave<VS>(a, j) : mk<double>(0.0, 0.0), pre, row);
    mstore<BL, 3>(mregion<BL>(a, kPartB + 1), a.geo.G, rr.lb, e);
}

// C-kernel: half-step test on ||s||; omega; x += alpha p + omega s;
// r = s - omega t; partials <rhat, r>, ||r||^2.
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_C(const MultiArgs a) {
    if (all_done(a)) return;
    HZ_MULTI_ROWS;
    double h[4], e[3] = {0.0, 0.0, 0.0};
    mhead<BL, 4>(mregion<BL>(a, kPartB), a.geo.G, h);
    int mode = 0;  // 0: nothing, 1: half-step exit, 2: full step
    double2 al = mk<double>(0.0, 0.0), om = mk<double>(0.0, 0.0);
    if (j < a.B) {
        SolverScal* sc = a.sc + j;
        const bool lead = mleader<BL>(rr.lb);
        // pending is written by this kernel's leader, so only done is read
        // here (a pending exit of the previous iteration was concluded by P)
        if (!sc->done) {
            const int it = sc->cur;
            const double rel = __builtin_sqrt(h[0]) / sc->bnorm;
            al = sc->alpha;
            if (!__builtin_isfinite(rel)) {
                if (lead) finish(sc, a.ndone, ST_NONFINITE, it);
            } else if (rel <= sc->rtol) {  // concluded by the next P-kernel
                mode = 1;
                if (lead) {
                    sc->relres = rel;
                    sc->pending = it;
                }
            } else {
                const double2 ts = mk<double>(h[1], h[2]);
                const double tt = h[3];
                int st = -1, why = BD_NONE;
                if (!zfinite(ts) || !__builtin_isfinite(tt)) st = ST_NONFINITE;
                else if (tt == 0.0) st = ST_BREAKDOWN, why = BD_TT;
                else {
                    om = zdiv(ts, mk<double>(tt, 0.0));
                    if (!zfinite(om)) st = ST_NONFINITE;
                }
                if (st >= 0) {
                    if (lead) finish(sc, a.ndone, st, it, why);
                } else {
                    mode = 2;
                    if (lead) {
                        sc->omega = om;
                        sc->iter = it + 1;
                    }
                }
            }
        }
    }
    if (mode == 1) {
        HZ_MROWS(i) {
            const size_t q = (size_t)i * Bz + j;
            a.x[q] = cfma<double>(al, a.p[q], a.x[q]);
        }
    } else if (mode == 2) {
        const double2 nom = mk<double>(-om.x, -om.y);
        HZ_MROWS(i) {
            const size_t q = (size_t)i * Bz + j;
            const double2 sv = a.s[q], tv = a.t[q], rh = a.rh[q];
            double2 x = a.x[q];
            x = cfma<double>(al, a.p[q], x);
            x = cfma<double>(om, sv, x);
            a.x[q] = x;
            const double2 r = cfma<double>(nom, tv, sv);
            a.r[q] = r;
            const double2 c = cdotacc(rh.x, rh.y, r.x, r.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
            e[2] = __builtin_fma(r.x, r.x, e[2]);
            e[2] = __builtin_fma(r.y, r.y, e[2]);
        }
    }
    mstore<BL, 3>(mregion<BL>(a, kPartC), a.geo.G, rr.lb, e);
}

// y = b - A xin for every system (explicit values `vals`, or K, M, Bm);
// partial ||y||^2 (I).
template <int BL, int U, int VS>
__global__ HZ_STREAM_BOUNDS void k_m_resid(const MultiArgs a, const double2* __restrict__ vals,
                                           const double2* __restrict__ xin, double2* __restrict__ y) {
    HZ_MULTI_ROWS;
    MultiArgs a2 = a;
    a2.vals = vals;
    double e[1] = {0.0};
    const double2 k = j < a.B ? mwave<VS>(a, j) : mk<double>(0.0, 0.0);
    auto pre = [&](int64_t i) { return a.b[(size_t)i * Bz + j]; };
    auto row = [&](int64_t i, double2 acc, double2 bv) {
        const double2 d = mk<double>(bv.x - acc.x, bv.y - acc.y);
        y[(size_t)i * Bz + j] = d;
        e[0] = __builtin_fma(d.x, d.x, e[0]);
        e[0] = __builtin_fma(d.y, d.y, e[0]);
    };
    m_tiles<BL, U, VS>(a2, rr, j < a.B, xin, k, pre, row);
    mstore<BL, 1>(mregion<BL>(a, kPartI), a.geo.G, rr.lb, e);
}

// relres_true of every system from region I (one block).
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_fin_true(const MultiArgs a) {
    double h[1];
    mhead<BL, 1>(mregion<BL>(a, kPartI), a.geo.G, h);
    const int j = threadIdx.x;
    if (j >= a.B) return;
    SolverScal* sc = a.sc + j;
    sc->relres_true = sc->bnorm > 0.0 ? __builtin_sqrt(h[0]) / sc->bnorm : 0.0;
}

// x = 0 for the systems whose right-hand side is zero.
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_zero_if(const MultiArgs a) {
    HZ_MULTI_ROWS;
    if (j >= a.B || !a.sc[j].zero_x) return;
    HZ_MROWS(i) a.x[(size_t)i * Bz + j] = mk<double>(0.0, 0.0);
}

// dinv[i*B + j] = 1 / A_j(i, i); a missing or zero diagonal flags sc[j].bad_diag.
__global__ __launch_bounds__(kBlock) void k_m_jacobi(int n, int B, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const double2* __restrict__ vals,
                                                     double2* __restrict__ dinv, SolverScal* sc) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= (int64_t)n * B) return;
    const int64_t i = f / B;
    const int j = (int)(f % B);
    double2 d = mk<double>(0.0, 0.0);
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = vals[(size_t)p * B + j];
    if (d.x == 0.0 && d.y == 0.0) {
        sc[j].bad_diag = 1;  // every writer stores 1
        dinv[f] = mk<double>(0.0, 0.0);
        return;
    }
    const double q = d.x * d.x + d.y * d.y;
    dinv[f] = mk<double>(d.x / q, -d.y / q);
}

// dinv[i*B + j] = 1 / (K_ii - k_j^2 M_ii + i k_j Bm_ii); a missing or zero
// diagonal flags sc[j].bad_diag.
__global__ __launch_bounds__(kBlock) void k_m_jacobi_kmb(int n, int B, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ K,
                                                         const double* __restrict__ M, const double* __restrict__ Bm,
                                                         const double* __restrict__ kw, double2* __restrict__ dinv,
                                                         SolverScal* sc) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= (int64_t)n * B) return;
    const int64_t i = f / B;
    const int j = (int)(f % B);
    const double kj = kw[j];
    double2 d = mk<double>(0.0, 0.0);
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = mk<double>(__builtin_fma(-kj * kj, M[p], K[p]), kj * Bm[p]);
    if (d.x == 0.0 && d.y == 0.0) {
        sc[j].bad_diag = 1;  // every writer stores 1
        dinv[f] = mk<double>(0.0, 0.0);
        return;
    }
    const double q = d.x * d.x + d.y * d.y;
    dinv[f] = mk<double>(d.x / q, -d.y / q);
}

// kd[4 i .. 4 i + 3] = (K_ii, M_ii, Bm_ii, 0): the last diagonal entry of row i
// (the one k_m_jacobi_kmb uses), zeros if the row has none.
__global__ __launch_bounds__(kBlock) void k_m_diag_kmb(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ K, const double* __restrict__ M,
                                                       const double* __restrict__ Bm, double* __restrict__ kd) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double k = 0.0, m = 0.0, b = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) k = K[p], m = M[p], b = Bm[p];
    reinterpret_cast<double2*>(kd)[2 * i] = mk<double>(k, m);
    reinterpret_cast<double2*>(kd)[2 * i + 1] = mk<double>(b, 0.0);
}

// out[p*B + j] = vals[p*B + j] * dinv[col_p*B + j]   (A_j D_j^{-1})
__global__ __launch_bounds__(kBlock) void k_m_colscale(int64_t nnz, int B, const int* __restrict__ ci,
                                                       const double2* __restrict__ vals,
                                                       const double2* __restrict__ dinv, double2* __restrict__ out) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nnz * B) return;
    const int64_t p = f / B;
    const int j = (int)(f % B);
    out[f] = cmul<double>(vals[f], dinv[(size_t)ci[p] * B + j]);
}

// Conjugate transposes of every system: tvals[q*B + j] = conj(vals[tsrc[q]*B + j]).
__global__ __launch_bounds__(kBlock) void k_m_conj_vals(int64_t nnz, int B, const int* __restrict__ tsrc,
                                                        const double2* __restrict__ vals,
                                                        double2* __restrict__ tvals) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nnz * B) return;
    const int64_t q = f / B;
    const int j = (int)(f % B);
    const double2 a = vals[(size_t)tsrc[q] * B + j];
    tvals[f] = mk<double>(a.x, -a.y);
}

// Entry gradients of every system: grad[p*B + j] = -lam_j[row_p] conj(x_j[col_p]).
template <int BL>
__global__ HZ_STREAM_BOUNDS void k_m_grad_vals(const MultiArgs a, const double2* __restrict__ lam,
                                               const double2* __restrict__ xs, double2* __restrict__ grad) {
    HZ_MULTI_ROWS;
    if (j >= a.B) return;
    HZ_MROWS(i) {
        const double2 l = lam[(size_t)i * Bz + j];
        const double2 nl = mk<double>(-l.x, -l.y);
        for (int p = a.row_ptr[i]; p < a.row_ptr[i + 1]; ++p) {
            const double2 xv = xs[(size_t)a.col_idx[p] * Bz + j];
            grad[(size_t)p * Bz + j] = cmul<double>(nl, mk<double>(xv.x, -xv.y));
        }
    }
}

// Columns of a system-minor [n][B] array for a group of Bg <= kSweepGroup
// systems: gather (dir 0) dst[i*Bg + k] = src[i*B + idx[k]], or scatter
// (dir 1) dst[i*B + idx[k]] = src[i*Bg + k].
constexpr int kSweepGroup = 16;
// Ordering key of system j for grouping a batch: the sum of Re(A_j(i, i))
// over up to kBlock evenly spaced rows i (duplicates of a diagonal entry
// all count; a row without one adds nothing), in a fixed order.  For a
// frequency sweep K - k^2 M + i k B it decreases with k.  One block per
// system.
__global__ __launch_bounds__(kBlock) void k_m_diag_key(int n, int B, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const double2* __restrict__ vals,
                                                       double* __restrict__ key) {
    __shared__ double red[kBlock];
    const int j = blockIdx.x, t = threadIdx.x;
    const int m = n < kBlock ? n : kBlock;
    double v = 0.0;
    if (t < m) {
        const int i = (int)((int64_t)t * n / m);
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) v += vals[(size_t)p * B + j].x;
    }
    red[t] = v;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w /= 2) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) key[j] = red[0];
}

struct GroupCols {
    int j[kSweepGroup];
};
__global__ __launch_bounds__(kBlock) void k_m_cols(int n, int B, int Bg, GroupCols idx, const double2* __restrict__ src,
                                                   double2* __restrict__ dst, int dir) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= (int64_t)n * Bg) return;
    const int64_t i = f / Bg;
    const int k = (int)(f % Bg);
    const int64_t w = i * B + idx.j[k];
    if (dir == 0) dst[f] = src[w];
    else dst[w] = src[f];
}

}  // namespace hz
