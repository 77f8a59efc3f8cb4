// Device kernels of the helmz library (gfx950 / CDNA4, wave64).
//
// Every kernel that reduces writes one fixed-order partial per block and a
// single-block kernel sums the partials in index order, so results are
// bitwise reproducible run to run (no floating-point atomics anywhere).
//
// Row ownership: a launch of G blocks splits the rows into G contiguous
// chunks.  Hardware dispatches block b to XCD (b mod 8); block b works on
// logical chunk (b mod 8) * (G/8) + b/8, so each XCD owns one contiguous
// eighth of the rows.  The x-gathers of a banded FE matrix then stay inside
// that XCD's L2, and every kernel of a solve maps the same rows to the same
// XCD.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hz {

constexpr int kWave = 64;
constexpr int kXcd = 8;
constexpr int kBlock = 256;
constexpr int kMaxGrid = 2048;  // bound on blocks (= partials) of a reducing launch
constexpr int kMaxParts = 4;    // components per partial

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
// conj(a) b, accumulated in double
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

// Block sum of K doubles; the result is valid in thread 0 only.  Waves are
// combined in a fixed order.
template <int K> __device__ __forceinline__ void block_sum(double (&v)[K]) {
    __shared__ double lds[kBlock / kWave][K];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = group_sum<64>(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wid][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = lds[0][k];
            for (int w = 1; w < kBlock / kWave; ++w) s += lds[w][k];
            v[k] = s;
        }
    }
}

// Sum K component arrays of G partials (component k at part[k*G + g]) in a
// fixed order: thread t adds g = t, t+256, ... sequentially, then block_sum.
template <int K> __device__ __forceinline__ void sum_partials(const double* __restrict__ part, int G, double (&out)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int g = threadIdx.x; g < G; g += kBlock) s += part[k * G + g];
        out[k] = s;
    }
    block_sum<K>(out);
}

// ------------------------------------------------------------------ launch geometry

// Chunked row ownership of a launch (see the file comment).
struct Geom {
    int G;      // blocks
    int chunk;  // rows per block, a multiple of the rows one block step covers
};

__device__ __forceinline__ int logical_block(int b, int G) {
    return (G % kXcd == 0) ? (b % kXcd) * (G / kXcd) + b / kXcd : b;
}

// ------------------------------------------------------------------ solver scalars (device resident)

struct alignas(256) SolverScal {
    double2 rho;    // <rhat, r> for the current iteration
    double2 alpha;  // rho / <rhat, v>
    double2 omega;  // <t, s> / <t, t>
    double2 beta;   // (rho_new / rho) (alpha / omega)
    double bnorm;   // ||b||
    double rtol;
    double relres;       // last recursive ||r|| / ||b|| (or ||s|| / ||b||)
    double relres_true;  // filled by the final residual check
    int iter;            // current iteration, 1-based
    int maxiter;
    int status;  // solver status once done
    int done;    // 1 once the solve has ended (all later kernels are no-ops)
    int half;    // the half step met the tolerance: x += alpha p and stop
    int first;   // iteration 1: p = r
    int zero_x;  // ||b|| = 0: the solution is x = 0
    int bad_diag;  // Jacobi requested with a zero diagonal entry
    double outer_rn;  // refinement: ||b - A x|| of the current outer step
};

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };

// Reset a scalar block before a solve (one thread).
__global__ void k_sc_init(SolverScal* sc, double rtol, int maxiter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    SolverScal z = {};
    z.rtol = rtol;
    z.maxiter = maxiter;
    z.status = 1;
    *sc = z;
}

__device__ __forceinline__ void finish(SolverScal* sc, int status, int iterations) {
    sc->status = status;
    sc->iter = iterations;
    sc->done = 1;
}

// ------------------------------------------------------------------ SpMV with fused epilogues

enum : int {
    EPI_NONE = 0,   // y = A x
    EPI_DOT_W = 1,  // y = A x;  partial conj(w_i) y_i            (2 comps)
    EPI_TS = 2,     // y = A x;  partials conj(y_i) x_i, |y_i|^2   (3 comps)
    EPI_RESID = 3   // y = w - A x; partial |y_i|^2                (1 comp)
};

template <typename T> struct SpmvArgs {
    int n;
    Geom geo;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const cx<T>* __restrict__ vals;
    const cx<T>* __restrict__ x;
    cx<T>* __restrict__ y;
    const cx<T>* __restrict__ w;  // rhat (EPI_DOT_W) or b (EPI_RESID)
    double* __restrict__ part;    // partials, component-major, stride geo.G
    const SolverScal* sc;         // skip when done (and, for EPI_TS, on a half-step exit); may be null
};

template <int EPI> constexpr int epi_parts() { return EPI == EPI_DOT_W ? 2 : EPI == EPI_TS ? 3 : EPI == EPI_RESID ? 1 : 0; }

// Vector CSR: L lanes per row, BLOCK/L rows per block step.  Lane l of a row
// handles entries beg+l, beg+l+L, ...; the row total is a DPP group sum.
template <typename T, int L, int EPI>
__global__ __launch_bounds__(kBlock) void k_spmv(const SpmvArgs<T> a) {
    if (a.sc != nullptr) {
        if (a.sc->done) return;
        if (EPI == EPI_TS && a.sc->half) return;
    }
    constexpr int RPS = kBlock / L;  // rows per block step
    constexpr int K = epi_parts<EPI>();
    const int lb = logical_block(blockIdx.x, a.geo.G);
    const int64_t r0 = (int64_t)lb * a.geo.chunk;
    const int64_t r1 = r0 + a.geo.chunk < (int64_t)a.n ? r0 + a.geo.chunk : (int64_t)a.n;
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    double e[K > 0 ? K : 1];
#pragma unroll
    for (int k = 0; k < (K > 0 ? K : 1); ++k) e[k] = 0.0;

    for (int64_t base = r0; base < r1; base += RPS) {  // uniform trip count in the block
        const int64_t row = base + g;
        const bool ok = row < r1;
        cx<T> acc = mk<T>(T(0), T(0));
        if (ok) {
            const int beg = a.row_ptr[row], end = a.row_ptr[row + 1];
            for (int p = beg + lane; p < end; p += L) acc = cfma<T>(a.vals[p], a.x[a.col_idx[p]], acc);
        }
        acc.x = group_sum<L>(acc.x);
        acc.y = group_sum<L>(acc.y);
        if (ok && lane == 0) {
            if constexpr (EPI == EPI_RESID) {
                const cx<T> bw = a.w[row];
                acc.x = bw.x - acc.x;
                acc.y = bw.y - acc.y;
                e[0] = __builtin_fma((double)acc.x, (double)acc.x, e[0]);
                e[0] = __builtin_fma((double)acc.y, (double)acc.y, e[0]);
            }
            a.y[row] = acc;
            if constexpr (EPI == EPI_DOT_W) {
                const cx<T> wv = a.w[row];
                double2 c = mk<double>(e[0], e[1]);
                c = cdotacc(wv.x, wv.y, acc.x, acc.y, c);
                e[0] = c.x;
                e[1] = c.y;
            }
            if constexpr (EPI == EPI_TS) {
                const cx<T> sv = a.x[row];
                double2 c = mk<double>(e[0], e[1]);
                c = cdotacc(acc.x, acc.y, sv.x, sv.y, c);
                e[0] = c.x;
                e[1] = c.y;
                e[2] = __builtin_fma((double)acc.x, (double)acc.x, e[2]);
                e[2] = __builtin_fma((double)acc.y, (double)acc.y, e[2]);
            }
        }
    }
    if constexpr (K > 0) {
        block_sum<K>(e);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) a.part[k * a.geo.G + lb] = e[k];
        }
    }
}

// ------------------------------------------------------------------ element-wise kernels

#define HZ_ROWS(a)                                                                           \
    const int lb = logical_block(blockIdx.x, (a).geo.G);                                     \
    const int64_t r0 = (int64_t)lb * (a).geo.chunk;                                          \
    const int64_t r1 = r0 + (a).geo.chunk < (int64_t)(a).n ? r0 + (a).geo.chunk : (int64_t)(a).n

template <typename T> struct VecArgs {
    int n;
    Geom geo;
    const cx<T>* __restrict__ a;
    const cx<T>* __restrict__ b;
    const cx<T>* __restrict__ c;
    cx<T>* __restrict__ o1;
    cx<T>* __restrict__ o2;
    const cx<T>* __restrict__ w;
    double* __restrict__ part;
    SolverScal* sc;
};

// p = r                       (first iteration)
// p = r + beta (p - omega v)  (otherwise)            a = r, c = v, o1 = p
template <typename T> __global__ __launch_bounds__(kBlock) void k_pupd(const VecArgs<T> a) {
    if (a.sc->done) return;
    HZ_ROWS(a);
    const bool first = a.sc->first != 0;
    const double2 bd = a.sc->beta, od = a.sc->omega;
    const cx<T> beta = mk<T>((T)bd.x, (T)bd.y), omega = mk<T>((T)od.x, (T)od.y);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const cx<T> r = a.a[i];
        if (first) {
            a.o1[i] = r;
        } else {
            const cx<T> p = a.o1[i], v = a.c[i];
            cx<T> d = mk<T>(p.x - fmaT(omega.x, v.x, -omega.y * v.y), p.y - fmaT(omega.x, v.y, omega.y * v.x));
            a.o1[i] = cfma<T>(beta, d, r);
        }
    }
}

// s = r - alpha v ; partial ||s||^2                  a = r, b = v, o1 = s
template <typename T> __global__ __launch_bounds__(kBlock) void k_supd(const VecArgs<T> a) {
    if (a.sc->done) return;
    HZ_ROWS(a);
    const double2 ad = a.sc->alpha;
    const cx<T> al = mk<T>((T)ad.x, (T)ad.y);
    double e[1] = {0.0};
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const cx<T> r = a.a[i], v = a.b[i];
        cx<T> s = cfma<T>(mk<T>(-al.x, -al.y), v, r);
        a.o1[i] = s;
        e[0] = __builtin_fma((double)s.x, (double)s.x, e[0]);
        e[0] = __builtin_fma((double)s.y, (double)s.y, e[0]);
    }
    block_sum<1>(e);
    if (threadIdx.x == 0) a.part[lb] = e[0];
}

// Full step: x += alpha p + omega s ; r = s - omega t ; partials conj(rhat) r, ||r||^2
// Half-step exit: x += alpha p only.      a = p, b = s, c = t, o1 = x, o2 = r, w = rhat
template <typename T> __global__ __launch_bounds__(kBlock) void k_xr(const VecArgs<T> a) {
    if (a.sc->done) return;
    HZ_ROWS(a);
    const double2 ad = a.sc->alpha, od = a.sc->omega;
    const cx<T> al = mk<T>((T)ad.x, (T)ad.y), om = mk<T>((T)od.x, (T)od.y);
    if (a.sc->half) {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) a.o1[i] = cfma<T>(al, a.a[i], a.o1[i]);
        return;
    }
    double e[3] = {0.0, 0.0, 0.0};
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const cx<T> p = a.a[i], s = a.b[i], t = a.c[i], rh = a.w[i];
        cx<T> x = a.o1[i];
        x = cfma<T>(al, p, x);
        x = cfma<T>(om, s, x);
        a.o1[i] = x;
        const cx<T> r = cfma<T>(mk<T>(-om.x, -om.y), t, s);
        a.o2[i] = r;
        double2 c = mk<double>(e[0], e[1]);
        c = cdotacc(rh.x, rh.y, r.x, r.y, c);
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma((double)r.x, (double)r.x, e[2]);
        e[2] = __builtin_fma((double)r.y, (double)r.y, e[2]);
    }
    block_sum<3>(e);
    if (threadIdx.x == 0) {
        a.part[lb] = e[0];
        a.part[a.geo.G + lb] = e[1];
        a.part[2 * a.geo.G + lb] = e[2];
    }
}

// Solve set-up: r = src, rhat = src; partials ||b||^2, ||r||^2.
// a = b, b = src (b itself, or the residual b - A x0), o1 = r, o2 = rhat
template <typename T> __global__ __launch_bounds__(kBlock) void k_init(const VecArgs<T> a) {
    HZ_ROWS(a);
    double e[2] = {0.0, 0.0};
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const cx<T> bv = a.a[i], r = a.b[i];
        if (a.o1 != a.b) a.o1[i] = r;
        a.o2[i] = r;
        e[0] = __builtin_fma((double)bv.x, (double)bv.x, e[0]);
        e[0] = __builtin_fma((double)bv.y, (double)bv.y, e[0]);
        e[1] = __builtin_fma((double)r.x, (double)r.x, e[1]);
        e[1] = __builtin_fma((double)r.y, (double)r.y, e[1]);
    }
    block_sum<2>(e);
    if (threadIdx.x == 0) {
        a.part[lb] = e[0];
        a.part[a.geo.G + lb] = e[1];
    }
}

// ------------------------------------------------------------------ single-block finalisers

__global__ __launch_bounds__(kBlock) void k_fin_init(const double* __restrict__ part, int G, SolverScal* sc) {
    double s[2];
    sum_partials<2>(part, G, s);
    if (threadIdx.x != 0) return;
    const double bn = __builtin_sqrt(s[0]);
    sc->bnorm = bn;
    sc->iter = 1;
    sc->first = 1;
    sc->half = 0;
    sc->done = 0;
    sc->zero_x = 0;
    sc->status = ST_NOT_CONVERGED;
    sc->rho = mk<double>(s[1], 0.0);
    sc->alpha = sc->omega = sc->beta = mk<double>(1.0, 0.0);
    if (!__builtin_isfinite(bn) || !__builtin_isfinite(s[1])) {
        finish(sc, ST_NONFINITE, 0);
        return;
    }
    if (bn == 0.0) {
        sc->zero_x = 1;
        sc->relres = 0.0;
        finish(sc, ST_OK, 0);
        return;
    }
    const double rel = __builtin_sqrt(s[1]) / bn;
    sc->relres = rel;
    if (rel <= sc->rtol) finish(sc, ST_OK, 0);
    else if (sc->maxiter <= 0) finish(sc, ST_NOT_CONVERGED, 0);
}

// alpha = rho / <rhat, v>
__global__ __launch_bounds__(kBlock) void k_fin_alpha(const double* __restrict__ part, int G, SolverScal* sc) {
    if (sc->done) return;
    double s[2];
    sum_partials<2>(part, G, s);
    if (threadIdx.x != 0) return;
    const double2 sigma = mk<double>(s[0], s[1]);
    if (!zfinite(sigma)) return finish(sc, ST_NONFINITE, sc->iter);
    if (zzero(sigma)) return finish(sc, ST_BREAKDOWN, sc->iter);
    sc->alpha = zdiv(sc->rho, sigma);
}

// half-step test on ||s||
__global__ __launch_bounds__(kBlock) void k_fin_half(const double* __restrict__ part, int G, SolverScal* sc) {
    if (sc->done) return;
    double s[1];
    sum_partials<1>(part, G, s);
    if (threadIdx.x != 0) return;
    const double rel = __builtin_sqrt(s[0]) / sc->bnorm;
    if (!__builtin_isfinite(rel)) return finish(sc, ST_NONFINITE, sc->iter);
    if (rel <= sc->rtol) {
        sc->relres = rel;
        sc->half = 1;
    }
}

// omega = <t, s> / <t, t>
__global__ __launch_bounds__(kBlock) void k_fin_omega(const double* __restrict__ part, int G, SolverScal* sc) {
    if (sc->done || sc->half) return;
    double s[3];
    sum_partials<3>(part, G, s);
    if (threadIdx.x != 0) return;
    const double2 ts = mk<double>(s[0], s[1]);
    const double tt = s[2];
    if (!zfinite(ts) || !__builtin_isfinite(tt)) return finish(sc, ST_NONFINITE, sc->iter);
    if (tt == 0.0) return finish(sc, ST_BREAKDOWN, sc->iter);
    const double2 om = zdiv(ts, mk<double>(tt, 0.0));
    if (!zfinite(om)) return finish(sc, ST_NONFINITE, sc->iter);
    sc->omega = om;
}

// end of an iteration: convergence on ||r||, breakdown tests, next rho and beta
__global__ __launch_bounds__(kBlock) void k_fin_rho(const double* __restrict__ part, int G, SolverScal* sc) {
    if (sc->done) return;
    if (sc->half) {  // x was updated with alpha p by k_xr
        if (threadIdx.x == 0) finish(sc, ST_OK, sc->iter);
        return;
    }
    double s[3];
    sum_partials<3>(part, G, s);
    if (threadIdx.x != 0) return;
    const int it = sc->iter;
    const double rel = __builtin_sqrt(s[2]) / sc->bnorm;
    sc->relres = rel;
    if (!__builtin_isfinite(rel)) return finish(sc, ST_NONFINITE, it);
    if (rel <= sc->rtol) return finish(sc, ST_OK, it);
    if (zzero(sc->omega)) return finish(sc, ST_BREAKDOWN, it);
    if (it >= sc->maxiter) return finish(sc, ST_NOT_CONVERGED, sc->maxiter);
    const double2 rho_new = mk<double>(s[0], s[1]);
    if (!zfinite(rho_new)) return finish(sc, ST_NONFINITE, it + 1);
    if (zzero(rho_new)) return finish(sc, ST_BREAKDOWN, it + 1);
    const double2 beta = zmul(zdiv(rho_new, sc->rho), zdiv(sc->alpha, sc->omega));
    if (!zfinite(beta)) return finish(sc, ST_NONFINITE, it + 1);
    sc->beta = beta;
    sc->rho = rho_new;
    sc->first = 0;
    sc->iter = it + 1;
}

// relres_true = sqrt(sum) / ||b||
__global__ __launch_bounds__(kBlock) void k_fin_true(const double* __restrict__ part, int G, SolverScal* sc) {
    double s[1];
    sum_partials<1>(part, G, s);
    if (threadIdx.x == 0) sc->relres_true = sc->bnorm > 0.0 ? __builtin_sqrt(s[0]) / sc->bnorm : 0.0;
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
        sc->bad_diag = 1;  // benign race: every writer stores 1
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_if(int n, const SolverScal* sc, cx<T>* __restrict__ x) {
    if (!sc->zero_x) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = mk<T>(T(0), T(0));
}

// ------------------------------------------------------------------ standalone BLAS-1

template <int MODE>  // 0: conj(x) y  (2 comps), 1: |x|^2 (1 comp)
__global__ __launch_bounds__(kBlock) void k_dot_part(int n, Geom geo, const double2* __restrict__ x,
                                                     const double2* __restrict__ y, double* __restrict__ part) {
    struct {
        int n;
        Geom geo;
    } a{n, geo};
    HZ_ROWS(a);
    constexpr int K = MODE == 0 ? 2 : 1;
    double e[K];
#pragma unroll
    for (int k = 0; k < K; ++k) e[k] = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
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
    block_sum<K>(e);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[k * geo.G + lb] = e[k];
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_dot_fin(const double* __restrict__ part, int G, void* out) {
    constexpr int K = MODE == 0 ? 2 : 1;
    double s[K];
    sum_partials<K>(part, G, s);
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
    sum_partials<1>(part, G, s);
    if (threadIdx.x == 0) sc->bnorm = __builtin_sqrt(s[0]);
}

// After r = b - A x: decide convergence; otherwise record ||r|| for the next correction.
__global__ __launch_bounds__(kBlock) void k_fin_outer(const double* __restrict__ part, int G, SolverScal* sc,
                                                      int outer, int max_outer) {
    double s[1];
    sum_partials<1>(part, G, s);
    if (threadIdx.x != 0) return;
    const double rn = __builtin_sqrt(s[0]), bn = sc->bnorm;
    sc->outer_rn = rn;
    if (!__builtin_isfinite(rn) || !__builtin_isfinite(bn)) return finish(sc, ST_NONFINITE, outer);
    if (bn == 0.0) {
        sc->zero_x = 1;
        sc->relres = 0.0;
        return finish(sc, ST_OK, outer);
    }
    const double rel = rn / bn;
    sc->relres = rel;
    sc->relres_true = rel;
    if (rel <= sc->rtol) return finish(sc, ST_OK, outer);
    if (outer >= max_outer) return finish(sc, ST_NOT_CONVERGED, outer);
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
