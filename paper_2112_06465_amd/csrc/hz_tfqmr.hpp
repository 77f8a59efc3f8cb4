// TFQMR: the paper's P-TFQMR (Section 7, iterative Krylov methods), Freund's
// transpose-free QMR in the form of Saad's book.  One system, on the
// one-system work map of the BiCGStab kernels, their device scalars
// (SolverScal: rho, alpha, bnorm, rtol, status ...) and partial regions.
//
// Full iteration k (half steps m = 2k - 2, even, and m + 1, odd), three
// launches:
//   K1 (element-wise): alpha = rho / <r~, v>; u' = u - alpha v;
//       w -= alpha A u; d = u + (theta_m^2 / alpha) eta_m d; partial ||w||^2
//   K2 (product): theta, c, tau, eta of half step m + 1 from ||w||; the
//       quasi-residual test (x += eta d and done when it passes); then
//       A u' and, per row: x += eta d, w -= alpha A u',
//       d = u' + (theta^2 / alpha) eta d; partials ||w||^2, <r~, w>
//   K3 (product): the same scalars for half step m + 2 and its tests;
//       beta = rho_new / rho; per gathered column u'' = w + beta u'
//       (formed on the fly); per row: x += eta d, u = u'', Au = A u'',
//       v = A u'' + beta (A u' + beta v); partial <r~, v>
// Above about 10^5 rows K3 runs as two launches (k_q_dir, k_q_next_light) so
// that its product gathers one vector, as the BiCGStab iteration does there.
// tau, theta, eta of half step m live in slot m & 1 of the TFQMR scalars,
// rho of iteration k in rho2[(k - 1) & 1]: a launch never reads a slot its
// own leader writes.  K1 reads the iteration number `iter` and publishes it
// as `cur`; K2 and K3 read `cur`, and K3 advances `iter`.  An exit found by
// K2 or K3 still needs every block's share of the last x update, so it is
// recorded (half_exit, end_exit) instead of ending the solve, and the next K1
// (or k_q_conclude after the last chunk) concludes it: a block that has not
// started when the leader writes the record must still do its rows.
#pragma once

#include "hz_kernels.hpp"

namespace hz {

struct TScal {
    double tau[2], theta[2];  // per half-step parity
    double2 eta[2];
    int half_exit;  // iteration whose first half step converged (0: none)
    int end_exit;   // iteration that ended at its second half step (0: none)
    int end_status, end_why;
};

struct QArgs {
    int G, stride;
    const BlockMap* bmap;
    const SysMap* smap;
    int* ndone;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col_idx;
    const double2* __restrict__ vals;
    const double2* rt;  // shadow residual r~
    double2* w;
    double2* u;    // u of the even half step (u'' after K3)
    double2* u1;   // u' = u - alpha v
    double2* au;   // A u
    double2* au1;  // A u'
    double2* v;
    double2* d;
    double2* x;
    double* part;
    SolverScal* sc;
    TScal* tq;
};

__device__ __forceinline__ SysBlock qblock(const QArgs& a) {
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

// theta, c, tau, eta of a half step from ||w||^2, the previous tau and alpha
struct QStep {
    double theta, tau;
    double2 eta;
};
__device__ __forceinline__ QStep q_step(double ww, double tau_prev, double2 alpha) {
    QStep st;
    st.theta = __builtin_sqrt(ww) / tau_prev;
    const double c2 = 1.0 / (1.0 + st.theta * st.theta);
    st.tau = tau_prev * st.theta * __builtin_sqrt(c2);
    st.eta = mk<double>(c2 * alpha.x, c2 * alpha.y);
    return st;
}

// (theta^2 / alpha) eta
__device__ __forceinline__ double2 q_dcoef(double theta, double2 eta, double2 alpha) {
    const double2 t = zdiv(eta, alpha);
    return mk<double>(theta * theta * t.x, theta * theta * t.y);
}

// TFQMR set-up: rho_0 = <r~, r_0>, tau_0 = ||r_0|| from the set-up partials
__global__ __launch_bounds__(kBlock) void k_q_fin_init(const QArgs a) {
    double h[3];
    const SysMap sm = a.smap[0];
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, sm.gbeg, sm.gcnt, h);
    if (threadIdx.x != 0) return;
    a.sc->rho2[0] = mk<double>(h[0], h[1]);
    a.tq->tau[0] = __builtin_sqrt(h[2]);
    a.tq->theta[0] = 0.0;
    a.tq->eta[0] = mk<double>(0.0, 0.0);
    a.tq->half_exit = 0;
    a.tq->end_exit = 0;
    a.tq->end_status = ST_NOT_CONVERGED;
    a.tq->end_why = BD_NONE;
}

// Leader of system 0: end the solve recorded by K2 or K3.  Returns whether
// one was recorded (then every block of the launch returns).
__device__ __forceinline__ bool q_conclude(const QArgs& a, bool leader) {
    const int he = a.tq->half_exit, ee = a.tq->end_exit;
    if (he == 0 && ee == 0) return false;
    if (leader) {
        if (he) finish(a.sc, a.ndone, ST_OK, he);
        else finish(a.sc, a.ndone, a.tq->end_status, ee, a.tq->end_why);
    }
    return true;
}

// After the last chunk: conclude an exit recorded by its last launches.
__global__ void k_q_conclude(const QArgs a) {
    if (a.sc->done) return;
    q_conclude(a, threadIdx.x == 0);
}

// A u_0 = A r_0: u = w = r_0, v = Au = A r_0, d = 0; partial <r~, v>
template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_q_init(const QArgs a, const double2* __restrict__ r0) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    double e[2] = {0.0, 0.0};
    for_rows<double, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, [r0](int c) { return r0[c]; },
                           [&](int64_t row, double2 acc) {
                               const double2 rv = r0[row];
                               a.u[row] = rv;
                               a.w[row] = rv;
                               a.au[row] = acc;
                               a.v[row] = acc;
                               a.d[row] = mk<double>(0.0, 0.0);
                               const double2 t = a.rt[row];
                               const double2 c = cdotacc(t.x, t.y, acc.x, acc.y, mk<double>(e[0], e[1]));
                               e[0] = c.x;
                               e[1] = c.y;
                           });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

// K1: the even half step's vector work
__global__ HZ_STREAM_BOUNDS void k_q_even(const QArgs a) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc;
    if (sc->done || q_conclude(a, sys_leader(q))) return;
    double h[2];
    sys_sum<2>(a.part + kPartA * a.stride, a.stride, q.gbeg, q.gcnt, h);
    const double2 sigma = mk<double>(h[0], h[1]);
    // the scalars are read after the reduction: held across it they spilled under the 64-register cap
    const int it = sc->iter;
    const double2 rho = sc->rho2[(it - 1) & 1];
    const double theta = a.tq->theta[0];
    const double2 eta = a.tq->eta[0];
    int st = -1, why = BD_NONE;
    double2 alpha = mk<double>(0.0, 0.0);
    if (!zfinite(sigma) || !zfinite(rho)) st = ST_NONFINITE;
    else if (zzero(sigma)) st = ST_BREAKDOWN, why = BD_RHAT_V;
    else if (zzero(rho)) st = ST_BREAKDOWN, why = BD_RHO;
    else {
        alpha = zdiv(rho, sigma);
        if (!zfinite(alpha)) st = ST_NONFINITE;
    }
    if (st >= 0) {
        if (sys_leader(q)) finish(sc, a.ndone, st, it - 1, why);
        return;
    }
    if (sys_leader(q)) {
        sc->alpha = alpha;
        sc->cur = it;
    }
    const double2 dc = q_dcoef(theta, eta, alpha), na = mk<double>(-alpha.x, -alpha.y);
    double e[1] = {0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        const double2 uv = a.u[i];
        a.u1[i] = cfma<double>(na, a.v[i], uv);
        const double2 wv = cfma<double>(na, a.au[i], a.w[i]);
        a.w[i] = wv;
        a.d[i] = cfma<double>(dc, a.d[i], uv);
        e[0] = __builtin_fma(wv.x, wv.x, e[0]);
        e[0] = __builtin_fma(wv.y, wv.y, e[0]);
    }
    store_sys_partials<1>(a.part + kPartB * a.stride, a.stride, q.lb, e);
}

// K2: the odd half step
template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_q_odd(const QArgs a) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc;
    if (sc->done) return;
    const int it = sc->cur;
    const double bnorm = sc->bnorm, rtol = sc->rtol, tau0 = a.tq->tau[0];
    const double2 alpha = sc->alpha;
    double h[1];
    sys_sum<1>(a.part + kPartB * a.stride, a.stride, q.gbeg, q.gcnt, h);
    const QStep s1 = q_step(h[0], tau0, alpha);
    const int m1 = 2 * it - 1;  // this half step's index + 1 (m + 1 with m = 2 it - 2)
    const double bound = __builtin_sqrt((double)(m1 + 1)) * s1.tau / bnorm;
    if (!__builtin_isfinite(bound)) {  // no block writes x: ending at once is safe
        if (sys_leader(q)) finish(sc, a.ndone, ST_NONFINITE, it);
        return;
    }
    if (bound <= rtol) {  // x_{m+1} = x_m + eta d solves: apply, and record a half-step exit
        HZ_FOR_ELEMS(i, q.rw) a.x[i] = cfma<double>(s1.eta, a.d[i], a.x[i]);
        if (sys_leader(q)) {
            sc->relres = bound;
            a.tq->half_exit = it;
        }
        return;
    }
    if (sys_leader(q)) {
        a.tq->tau[1] = s1.tau;
        a.tq->theta[1] = s1.theta;
        a.tq->eta[1] = s1.eta;
        sc->relres = bound;
    }
    const double2 dc = q_dcoef(s1.theta, s1.eta, alpha), na = mk<double>(-alpha.x, -alpha.y);
    const double2* __restrict__ u1 = a.u1;
    double e[3] = {0.0, 0.0, 0.0};
    for_rows<double, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, [u1](int c) { return u1[c]; },
                           [&](int64_t row, double2 acc) {
                               double2 dv = a.d[row];
                               a.x[row] = cfma<double>(s1.eta, dv, a.x[row]);
                               const double2 wv = cfma<double>(na, acc, a.w[row]);
                               a.w[row] = wv;
                               a.d[row] = cfma<double>(dc, dv, u1[row]);
                               a.au1[row] = acc;
                               e[0] = __builtin_fma(wv.x, wv.x, e[0]);
                               e[0] = __builtin_fma(wv.y, wv.y, e[0]);
                               const double2 t = a.rt[row];
                               const double2 c = cdotacc(t.x, t.y, wv.x, wv.y, mk<double>(e[1], e[2]));
                               e[1] = c.x;
                               e[2] = c.y;
                           });
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
}

// K3: the end of the odd half step and the next even step's directions
template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_q_next(const QArgs a) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc;
    if (sc->done || a.tq->half_exit) return;
    const int it = sc->cur;
    const double bnorm = sc->bnorm, rtol = sc->rtol, tau1 = a.tq->tau[1];
    const int maxit = sc->maxiter;
    const double2 alpha = sc->alpha, rho_old = sc->rho2[(it - 1) & 1];
    double h[3];
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, q.gbeg, q.gcnt, h);
    const QStep s2 = q_step(h[0], tau1, alpha);
    const double2 rho_new = mk<double>(h[1], h[2]);
    const int m2 = 2 * it;  // half step index + 1 of the iterate this launch completes
    const double bound = __builtin_sqrt((double)(m2 + 1)) * s2.tau / bnorm;
    int st = -1, why = BD_NONE;
    double2 beta = mk<double>(0.0, 0.0);
    if (!__builtin_isfinite(bound) || !zfinite(rho_new)) st = ST_NONFINITE;
    else if (bound <= rtol) st = ST_OK;
    else if (it >= maxit) st = ST_NOT_CONVERGED;
    else if (zzero(rho_old)) st = ST_BREAKDOWN, why = BD_RHO;
    else {
        beta = zdiv(rho_new, rho_old);
        if (!zfinite(beta)) st = ST_NONFINITE;
    }
    if (st >= 0) {  // x_{m+2} = x_{m+1} + eta d is the last iterate; the next K1 ends the solve
        if (st != ST_NONFINITE) HZ_FOR_ELEMS(i, q.rw) a.x[i] = cfma<double>(s2.eta, a.d[i], a.x[i]);
        if (sys_leader(q)) {
            sc->relres = bound;
            a.tq->end_status = st;
            a.tq->end_why = why;
            a.tq->end_exit = it;
        }
        return;
    }
    if (sys_leader(q)) {
        a.tq->tau[0] = s2.tau;
        a.tq->theta[0] = s2.theta;
        a.tq->eta[0] = s2.eta;
        sc->rho2[it & 1] = rho_new;
        sc->relres = bound;
        sc->iter = it + 1;
        sc->iters = it;
    }
    const double2* __restrict__ w = a.w;
    const double2* __restrict__ u1 = a.u1;
    auto ucol = [w, u1, beta](int c) { return cfma<double>(beta, u1[c], w[c]); };
    double e[2] = {0.0, 0.0};
    for_rows<double, L, U, false>(q.rw, a.row_ptr, a.col_idx, a.vals, ucol, [&](int64_t row, double2 acc) {
        a.x[row] = cfma<double>(s2.eta, a.d[row], a.x[row]);
        a.u[row] = ucol((int)row);
        a.au[row] = acc;
        const double2 inner = cfma<double>(beta, a.v[row], a.au1[row]);  // A u' + beta v
        const double2 vv = cfma<double>(beta, inner, acc);
        a.v[row] = vv;
        const double2 t = a.rt[row];
        const double2 c = cdotacc(t.x, t.y, vv.x, vv.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
    });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

// Gather-light form of K3 for large systems (two launches instead of one,
// one gathered vector instead of two): K3a takes the scalars, tests and exit
// records of K3 and forms u'' = w + beta u' and x += eta d element-wise;
// K3b gathers u'' alone for A u'' and updates Au, v and the <r~, v>
// partials.  Same arithmetic per element as K3.
__global__ HZ_STREAM_BOUNDS void k_q_dir(const QArgs a) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc;
    if (sc->done || a.tq->half_exit) return;
    const int it = sc->cur;
    const double bnorm = sc->bnorm, rtol = sc->rtol, tau1 = a.tq->tau[1];
    const int maxit = sc->maxiter;
    const double2 alpha = sc->alpha, rho_old = sc->rho2[(it - 1) & 1];
    double h[3];
    sys_sum<3>(a.part + kPartC * a.stride, a.stride, q.gbeg, q.gcnt, h);
    const QStep s2 = q_step(h[0], tau1, alpha);
    const double2 rho_new = mk<double>(h[1], h[2]);
    const double bound = __builtin_sqrt((double)(2 * it + 1)) * s2.tau / bnorm;
    int st = -1, why = BD_NONE;
    double2 beta = mk<double>(0.0, 0.0);
    if (!__builtin_isfinite(bound) || !zfinite(rho_new)) st = ST_NONFINITE;
    else if (bound <= rtol) st = ST_OK;
    else if (it >= maxit) st = ST_NOT_CONVERGED;
    else if (zzero(rho_old)) st = ST_BREAKDOWN, why = BD_RHO;
    else {
        beta = zdiv(rho_new, rho_old);
        if (!zfinite(beta)) st = ST_NONFINITE;
    }
    if (st >= 0) {
        if (st != ST_NONFINITE) HZ_FOR_ELEMS(i, q.rw) a.x[i] = cfma<double>(s2.eta, a.d[i], a.x[i]);
        if (sys_leader(q)) {
            sc->relres = bound;
            a.tq->end_status = st;
            a.tq->end_why = why;
            a.tq->end_exit = it;
        }
        return;
    }
    if (sys_leader(q)) {
        a.tq->tau[0] = s2.tau;
        a.tq->theta[0] = s2.theta;
        a.tq->eta[0] = s2.eta;
        sc->rho2[it & 1] = rho_new;
        sc->beta = beta;
        sc->relres = bound;
        sc->iter = it + 1;
        sc->iters = it;
    }
    HZ_FOR_ELEMS(i, q.rw) {
        a.x[i] = cfma<double>(s2.eta, a.d[i], a.x[i]);
        a.u[i] = cfma<double>(beta, a.u1[i], a.w[i]);
    }
}

template <int L, int U>
__global__ HZ_STREAM_BOUNDS void k_q_next_light(const QArgs a) {
    const SysBlock q = qblock(a);
    if (q.sys < 0) return;
    SolverScal* sc = a.sc;
    if (sc->done || a.tq->half_exit || a.tq->end_exit) return;
    const double2 beta = sc->beta;
    const double2* __restrict__ u = a.u;
    double e[2] = {0.0, 0.0};
    for_rows<double, L, U>(q.rw, a.row_ptr, a.col_idx, a.vals, [u](int c) { return u[c]; },
                           [&](int64_t row, double2 acc) {
                               a.au[row] = acc;
                               const double2 inner = cfma<double>(beta, a.v[row], a.au1[row]);
                               const double2 vv = cfma<double>(beta, inner, acc);
                               a.v[row] = vv;
                               const double2 t = a.rt[row];
                               const double2 c = cdotacc(t.x, t.y, vv.x, vv.y, mk<double>(e[0], e[1]));
                               e[0] = c.x;
                               e[1] = c.y;
                           });
    store_sys_partials<2>(a.part + kPartA * a.stride, a.stride, q.lb, e);
}

}  // namespace hz
