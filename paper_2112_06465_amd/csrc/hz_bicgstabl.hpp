// BiCGstab(l): the paper's P-BiCGSTAB(l) (Section 7, iterative Krylov
// methods; l = 8 in its speed-up tables), in the form of Sleijpen and
// Fokkema.  One system, on the one-system work map of the BiCGStab kernels
// and with the same device scalars (SolverScal) and partial regions.
//
// A cycle is l Bi-CG steps, each four launches (step j = 0 .. l-1):
//   U : rho_1 = <r~, r_j> (partials from the previous launch); at j = 0 the
//       cycle's convergence test on ||r_0|| and rho_0 = -omega rho_0;
//       beta = alpha rho_1 / rho_0; u_i = r_i - beta u_i (i <= j)
//   AU: u_{j+1} = A u_j; partial <r~, u_{j+1}>
//   R : alpha = rho_1 / <r~, u_{j+1}>; r_i -= alpha u_{i+1} (i <= j); x += alpha u_0
//   AR: r_{j+1} = A r_j; partial <r~, r_{j+1}> (rho of step j + 1)
// then the minimal-residual part, three launches:
//   gram  : partials of G_pq = <r_p, r_q>, 0 <= p <= q <= l
//   mr    : one block sums them and solves the normal equations
//           (R^H R) gamma = R^H r_0 (R = [r_1 .. r_l]) by Cholesky after
//           scaling to unit diagonal; omega = gamma_l
//   update: x += sum_j gamma_j r_{j-1}; r_0 -= sum_j gamma_j r_j;
//           u_0 -= sum_j gamma_j u_j; partials <r~, r_0>, ||r_0||^2
// ("A" is the column-scaled matrix under Jacobi, as for BiCGStab).  rho of
// global step s = (cycle - 1) l + j lives in rho2[s & 1]: the U-launch of
// step s reads slot (s - 1) & 1 and writes slot s & 1, which no block of the
// same launch reads.
#pragma once

#include "hz_kernels.hpp"
#include "hz_soltile.hpp"

namespace hz {

constexpr int kLMax = 8;                                   // largest l
constexpr int kGramPairs = (kLMax + 1) * (kLMax + 2) / 2;  // pairs p <= q of r_0 .. r_l
constexpr int kGramBlock = 256;                            // threads of a Gram block
constexpr int kGramMaxGrid = 256;                          // Gram blocks: one per CU
enum : int { BD_MR = 5 };                                  // the minimal-residual system is singular

struct LArgs {
    int G, stride;  // one-system map of the solver launches
    const BlockMap* bmap;
    const SysMap* smap;
    int* ndone;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const double2* __restrict__ vals;
    const double2* rt;  // shadow residual r~
    double2* r[kLMax + 1];
    double2* u[kLMax + 1];
    double2* x;       // iterate of the (column-scaled) system
    double* part;     // kParts x stride (regions as for BiCGStab)
    double* gpart;    // Gram partials: component c of block g at [c * kGramMaxGrid + g]
    double2* gam;     // gamma_1 .. gamma_l at [1 .. l]
    SolverScal* sc;
    int n, ell, j;    // rows, l, the Bi-CG step of this launch
    int gG;           // blocks of the Gram launch
    int pf = 1;       // partial slots per block that AU and AR write (sol_subs(G) when they run as sub-blocks)
};

__device__ __forceinline__ SysBlock lblock(const LArgs& a) {
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

__device__ __forceinline__ double2 zneg_mul(double2 a, double2 b) {  // -(a b)
    return mk<double>(-(a.x * b.x - a.y * b.y), -(a.x * b.y + a.y * b.x));
}

// U: beta, u_i = r_i - beta u_i (i <= j)
__global__ HZ_STREAM_BOUNDS void k_l_U(const LArgs a) {
    const SysBlock q = lblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc + q.sys;
    if (sc->done) return;
    const int it = sc->iter;  // cycle (1-based)
    const int s = (it - 1) * a.ell + a.j;
    const double bnorm = sc->bnorm, rtol = sc->rtol;
    const int maxc = sc->maxiter;
    const double2 alpha = sc->alpha, omega = sc->omega;
    const double2 rho_prev = s == 0 ? mk<double>(1.0, 0.0) : sc->rho2[(s + 1) & 1];
    double h[3];
    const int pf = a.j > 0 ? a.pf : 1;  // region C from AR (step j - 1), or from the update / set-up (j = 0)
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, pf * q.gbeg, pf * q.gcnt, h);
    const double2 rho1 = mk<double>(h[0], h[1]);
    double2 rho0 = rho_prev;
    if (a.j == 0) {  // a cycle starts: test the residual of the previous one
        const double rel = __builtin_sqrt(h[2]) / bnorm;
        int st = -1;
        if (!__builtin_isfinite(rel)) st = ST_NONFINITE;
        else if (rel <= rtol) st = ST_OK;
        else if (it - 1 >= maxc) st = ST_NOT_CONVERGED;
        if (sys_leader(q)) {
            sc->relres = rel;
            sc->cur = it;
        }
        if (st >= 0) {
            if (sys_leader(q)) finish(sc, a.ndone, st, it - 1);
            return;
        }
        rho0 = zneg_mul(omega, rho_prev);
    }
    int st = -1, why = BD_NONE;
    double2 beta = mk<double>(0.0, 0.0);
    if (!zfinite(rho1)) st = ST_NONFINITE;
    else if (zzero(rho0) || zzero(rho1)) st = ST_BREAKDOWN, why = BD_RHO;
    else {
        beta = zmul(alpha, zdiv(rho1, rho0));
        if (!zfinite(beta)) st = ST_NONFINITE;
    }
    if (st >= 0) {
        if (sys_leader(q)) finish(sc, a.ndone, st, it - 1, why);
        return;
    }
    if (sys_leader(q)) sc->rho2[s & 1] = rho1;
    const double2 nb = mk<double>(-beta.x, -beta.y);
    HZ_FOR_ELEMS(i, q.rw) {
        for (int p = 0; p <= a.j; ++p) a.u[p][i] = cfma<double>(nb, a.u[p][i], a.r[p][i]);
    }
}

// AU: u_{j+1} = A u_j; partial <r~, u_{j+1}>
template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_l_AU(const LArgs a) {
    const SysBlock q = lblock(a);
    if (q.sys < 0 || a.sc[q.sys].done) return;
    const double2* __restrict__ uj = a.u[a.j];
    double2* __restrict__ un = a.u[a.j + 1];
    const double2* __restrict__ rt = a.rt;
    double e[2] = {0.0, 0.0};
    for_rows<double, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, [uj](int c) { return uj[c]; },
                           [&](int64_t row, double2 acc) {
                               un[row] = acc;
                               const double2 w = rt[row];
                               const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
                               e[0] = c.x;
                               e[1] = c.y;
                           });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

// R: alpha, r_i -= alpha u_{i+1} (i <= j), x += alpha u_0
__global__ HZ_STREAM_BOUNDS void k_l_R(const LArgs a) {
    const SysBlock q = lblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc + q.sys;
    if (sc->done) return;
    const int it = sc->iter;
    const int s = (it - 1) * a.ell + a.j;
    const double2 rho1 = sc->rho2[s & 1];
    double h[2];
    sys_sum<2>(a.part + kPartA * a.stride, a.stride, a.pf * q.gbeg, a.pf * q.gcnt, h);
    const double2 g = mk<double>(h[0], h[1]);
    int st = -1, why = BD_NONE;
    double2 alpha = mk<double>(0.0, 0.0);
    if (!zfinite(g)) st = ST_NONFINITE;
    else if (zzero(g)) st = ST_BREAKDOWN, why = BD_RHAT_V;
    else {
        alpha = zdiv(rho1, g);
        if (!zfinite(alpha)) st = ST_NONFINITE;
    }
    if (st >= 0) {
        if (sys_leader(q)) finish(sc, a.ndone, st, it - 1, why);
        return;
    }
    if (sys_leader(q)) sc->alpha = alpha;
    const double2 na = mk<double>(-alpha.x, -alpha.y);
    HZ_FOR_ELEMS(i, q.rw) {
        for (int p = 0; p <= a.j; ++p) a.r[p][i] = cfma<double>(na, a.u[p + 1][i], a.r[p][i]);
        a.x[i] = cfma<double>(alpha, a.u[0][i], a.x[i]);
    }
}

// AR: r_{j+1} = A r_j; partial <r~, r_{j+1}> (the rho of the next step)
template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_l_AR(const LArgs a) {
    const SysBlock q = lblock(a);
    if (q.sys < 0 || a.sc[q.sys].done) return;
    const double2* __restrict__ rj = a.r[a.j];
    double2* __restrict__ rn = a.r[a.j + 1];
    const double2* __restrict__ rt = a.rt;
    double e[3] = {0.0, 0.0, 0.0};  // the norm slot is unused before the cycle's end
    for_rows<double, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, [rj](int c) { return rj[c]; },
                           [&](int64_t row, double2 acc) {
                               rn[row] = acc;
                               const double2 w = rt[row];
                               const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
                               e[0] = c.x;
                               e[1] = c.y;
                           });
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
}

// AU and AR on a large system: the tile loop of the standalone product as
// pf = sol_subs(G) blocks of kSpBlock threads per block of the map (r~ loaded with the
// tile, the product held in the LDS ring), one partial slot per sub-block.
__global__ __launch_bounds__(kSpBlock) void k_l_AUt(const LArgs a) {
    const SubBlock q = sub_block_of(a.bmap, a.G, a.pf);
    if (q.sys < 0 || a.sc[q.sys].done) return;
    const double2* __restrict__ uj = a.u[a.j];
    double2* __restrict__ un = a.u[a.j + 1];
    const double2* __restrict__ rt = a.rt;
    double e[2] = {0.0, 0.0};
    tile_loop<double, kHold>(
        q.rw, a.row_ptr, a.col_idx, a.vals, [uj](int c) { return uj[c]; }, [rt](int64_t row) { return rt[row]; },
        [&](int64_t, double2 acc, double2 w) {
            const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        },
        [un](int64_t row, double2 acc) { un[row] = acc; });
    store_sub_partials<2>(a.part + kPartA * a.stride, a.stride, q.ls, e);
}

__global__ __launch_bounds__(kSpBlock) void k_l_ARt(const LArgs a) {
    const SubBlock q = sub_block_of(a.bmap, a.G, a.pf);
    if (q.sys < 0 || a.sc[q.sys].done) return;
    const double2* __restrict__ rj = a.r[a.j];
    double2* __restrict__ rn = a.r[a.j + 1];
    const double2* __restrict__ rt = a.rt;
    double e[3] = {0.0, 0.0, 0.0};  // the norm slot is unused before the cycle's end
    tile_loop<double, kHold>(
        q.rw, a.row_ptr, a.col_idx, a.vals, [rj](int c) { return rj[c]; }, [rt](int64_t row) { return rt[row]; },
        [&](int64_t, double2 acc, double2 w) {
            const double2 c = cdotacc(w.x, w.y, acc.x, acc.y, mk<double>(e[0], e[1]));
            e[0] = c.x;
            e[1] = c.y;
        },
        [rn](int64_t row, double2 acc) { rn[row] = acc; });
    store_sub_partials<3>(a.part + kPartC * a.stride, a.stride, q.ls, e);
}

// Gram partials of <r_p, r_q>, 0 <= p <= q <= ELL, pair index in row-major
// order of the upper triangle; each of the gG blocks sums a contiguous chunk
// of rows in a fixed order.
template <int ELL>
__global__ __launch_bounds__(kGramBlock) void k_l_gram(const LArgs a) {
    constexpr int NP = (ELL + 1) * (ELL + 2) / 2;
    if (a.sc->done) return;  // uniform: one system
    double acc[2 * NP];
#pragma unroll
    for (int c = 0; c < 2 * NP; ++c) acc[c] = 0.0;
    const int64_t chunk = ((int64_t)a.n + a.gG - 1) / a.gG;
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < a.n ? i0 + chunk : a.n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kGramBlock) {
        double2 v[ELL + 1];
#pragma unroll
        for (int p = 0; p <= ELL; ++p) v[p] = a.r[p][i];
        int c = 0;
#pragma unroll
        for (int p = 0; p <= ELL; ++p)
#pragma unroll
            for (int qq = p; qq <= ELL; ++qq, ++c) {
                const double2 d = cdotacc(v[p].x, v[p].y, v[qq].x, v[qq].y, mk<double>(acc[2 * c], acc[2 * c + 1]));
                acc[2 * c] = d.x;
                acc[2 * c + 1] = d.y;
            }
    }
    __shared__ double lds[kGramBlock / kWave][2 * NP];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int c = 0; c < 2 * NP; ++c) {
        const double v = group_sum<64>(acc[c]);
        if (lane == 0) lds[wid][c] = v;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < 2 * NP; c += kGramBlock) {
        double sum = lds[0][c];
        for (int w = 1; w < kGramBlock / kWave; ++w) sum += lds[w][c];
        a.gpart[(int64_t)c * kGramMaxGrid + blockIdx.x] = sum;
    }
}

// One block: the Gram matrix, then the minimal-residual coefficients by
// Cholesky of the unit-diagonal scaled normal equations (thread 0).  Each
// Gram component is summed over the Gram blocks by an aligned group of 8
// lanes (lane l takes blocks l, l + 8, ...; then a DPP group sum), a fixed
// order.
template <int ELL>
__device__ __forceinline__ double2 gram_at(const double* g, int p, int qq) {  // <r_p, r_q>, any p, q
    const bool sw = p > qq;
    const int lo = sw ? qq : p, hi = sw ? p : qq;
    const int c = lo * (ELL + 1) - lo * (lo - 1) / 2 + (hi - lo);
    return mk<double>(g[2 * c], sw ? -g[2 * c + 1] : g[2 * c + 1]);
}

template <int ELL>
__global__ __launch_bounds__(kBlock) void k_l_mr(const LArgs a) {
    constexpr int NP = (ELL + 1) * (ELL + 2) / 2;
    static_assert(2 * NP * 8 <= kBlock, "8 lanes per Gram component");
    SolverScal* sc = a.sc;
    if (sc->done) return;  // uniform: one system
    __shared__ double g[2 * NP];
    __shared__ double2 L[ELL][ELL];
    __shared__ double2 y[ELL];
    __shared__ double d[ELL];
    {
        const int c = threadIdx.x / 8, l = threadIdx.x % 8;
        double sum = 0.0;
        if (c < 2 * NP) {
#pragma unroll 4
            for (int b = l; b < a.gG; b += 8) sum += a.gpart[(int64_t)c * kGramMaxGrid + b];
        }
        sum = group_sum<8>(sum);
        if (c < 2 * NP && l == 0) g[c] = sum;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int it = sc->iter;
    // scaled system: M'_pq = d_p G_pq d_q, c'_p = d_p <r_p, r_0>, d_p = 1 / sqrt(G_pp), p, q = 1 .. ELL
    bool ok = true;
    for (int p = 0; p < ELL; ++p) {
        const double gpp = gram_at<ELL>(g, p + 1, p + 1).x;
        ok = ok && __builtin_isfinite(gpp) && gpp > 0.0;
        d[p] = ok ? 1.0 / __builtin_sqrt(gpp) : 0.0;
    }
#pragma unroll 1
    for (int p = 0; p < ELL && ok; ++p)
#pragma unroll 1
        for (int qq = 0; qq <= p; ++qq) {  // lower Cholesky factor: M' = L L^H
            double2 sum = gram_at<ELL>(g, p + 1, qq + 1);
            sum = mk<double>(sum.x * d[p] * d[qq], sum.y * d[p] * d[qq]);
#pragma unroll 1
            for (int k = 0; k < qq; ++k) {  // sum -= L_pk conj(L_qk)
                const double2 l1 = L[p][k], l2 = L[qq][k];
                sum.x -= l1.x * l2.x + l1.y * l2.y;
                sum.y -= l1.y * l2.x - l1.x * l2.y;
            }
            if (p == qq) {
                ok = ok && __builtin_isfinite(sum.x) && sum.x > 0.0;
                L[p][p] = mk<double>(ok ? __builtin_sqrt(sum.x) : 0.0, 0.0);
            } else {
                L[p][qq] = mk<double>(sum.x / L[qq][qq].x, sum.y / L[qq][qq].x);
            }
        }
    if (!ok) {
        finish(sc, a.ndone, ST_BREAKDOWN, it - 1, BD_MR);
        return;
    }
#pragma unroll 1
    for (int p = 0; p < ELL; ++p) {  // L z = c'
        double2 sum = gram_at<ELL>(g, p + 1, 0);
        sum = mk<double>(sum.x * d[p], sum.y * d[p]);
#pragma unroll 1
        for (int k = 0; k < p; ++k) {
            const double2 t = zmul(L[p][k], y[k]);
            sum.x -= t.x;
            sum.y -= t.y;
        }
        y[p] = mk<double>(sum.x / L[p][p].x, sum.y / L[p][p].x);
    }
#pragma unroll 1
    for (int p = ELL - 1; p >= 0; --p) {  // L^H gamma' = z, gamma = D gamma'
        double2 sum = y[p];
#pragma unroll 1
        for (int k = p + 1; k < ELL; ++k) {  // (L^H)_pk = conj(L_kp)
            const double2 l = L[k][p], z = y[k];
            sum.x -= l.x * z.x + l.y * z.y;
            sum.y -= l.x * z.y - l.y * z.x;
        }
        y[p] = mk<double>(sum.x / L[p][p].x, sum.y / L[p][p].x);
    }
    bool fin = true;
    for (int p = 0; p < ELL; ++p) {
        const double2 gm = mk<double>(y[p].x * d[p], y[p].y * d[p]);
        fin = fin && zfinite(gm);
        a.gam[p + 1] = gm;
    }
    if (!fin) {
        finish(sc, a.ndone, ST_NONFINITE, it - 1);
        return;
    }
    const double2 om = a.gam[ELL];
    if (zzero(om)) {
        finish(sc, a.ndone, ST_BREAKDOWN, it, BD_OMEGA);
        return;
    }
    sc->omega = om;
    sc->iter = it + 1;
    sc->iters = it;
}

// update: x += sum gamma_j r_{j-1}; r_0 -= sum gamma_j r_j; u_0 -= sum gamma_j u_j;
// partials <r~, r_0>, ||r_0||^2 for the next cycle's first step
__global__ HZ_STREAM_BOUNDS void k_l_update(const LArgs a) {
    const SysBlock q = lblock(a);
    if (q.sys < 0 || a.sc[q.sys].done) return;
    double e[3] = {0.0, 0.0, 0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        double2 prev = a.r[0][i];
        double2 x = a.x[i], r0 = prev, u0 = a.u[0][i];
        for (int p = 1; p <= a.ell; ++p) {
            const double2 gm = a.gam[p], ng = mk<double>(-gm.x, -gm.y);  // uniform: scalar loads
            const double2 rp = a.r[p][i];
            x = cfma<double>(gm, prev, x);
            r0 = cfma<double>(ng, rp, r0);
            u0 = cfma<double>(ng, a.u[p][i], u0);
            prev = rp;
        }
        a.x[i] = x;
        a.r[0][i] = r0;
        a.u[0][i] = u0;
        const double2 w = a.rt[i];
        const double2 c = cdotacc(w.x, w.y, r0.x, r0.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma(r0.x, r0.x, e[2]);
        e[2] = __builtin_fma(r0.y, r0.y, e[2]);
    }
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
}

}  // namespace hz
