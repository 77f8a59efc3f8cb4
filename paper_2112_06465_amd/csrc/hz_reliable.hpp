// Mixed precision with reliable updates.
//
// The refinement of zbicgstab_solve_mixed restarts a complex64 BiCGStab for
// every correction, and each restart throws the Krylov space away.  This
// variant keeps one complex64 BiCGStab running on the scaled problem
// A D^{-1} y = b / ||b||, accumulates its iterate y in complex64, and every
// time its recursive residual has fallen by a factor delta (or the inner
// iteration has ended) performs a reliable update (Sleijpen and van der
// Vorst, reliable updated residuals in hybrid Bi-CG methods): the FP64
// iterate takes x += ||b|| D^{-1} y and y restarts from zero, the true
// residual r64 = b - A x is formed in FP64, and the complex64 recursive
// residual is replaced by r64 / ||b|| (with its <rhat, r>, ||r||^2 partials)
// while p, v, rhat and the scalars carry on.  Convergence is decided on the
// FP64 true residual only.
#pragma once

#include "hz_kernels.hpp"

namespace hz {

// out = in / ||b||  (complex64), ||b|| from the outer scalars
__global__ __launch_bounds__(kBlock) void k_ru_demote(int n, const double2* __restrict__ in, const SolverScal* sc,
                                                      float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / sc->bnorm;
    const double2 v = in[i];
    out[i] = mk<float>((float)(v.x * inv), (float)(v.y * inv));
}

// x += ||b|| D^{-1} y in FP64 (D^{-1} as the complex64 operator uses it), then y = 0
__global__ __launch_bounds__(kBlock) void k_ru_promote(int n, float2* __restrict__ y, const float2* __restrict__ dinv,
                                                       const SolverScal* sc, double2* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double bn = sc->bnorm;
    double2 d = mk<double>((double)y[i].x, (double)y[i].y);
    if (dinv != nullptr) d = zmul(mk<double>((double)dinv[i].x, (double)dinv[i].y), d);
    double2 xv = x[i];
    xv.x = __builtin_fma(bn, d.x, xv.x);
    xv.y = __builtin_fma(bn, d.y, xv.y);
    x[i] = xv;
    y[i] = mk<float>(0.0f, 0.0f);
}

// Replace the complex64 recursive residual by r64 / ||b|| and recompute the
// partials the next iteration starts from: <rhat, r>, ||r||^2 (region C).
__global__ HZ_STREAM_BOUNDS void k_ru_replace(const BicgArgs<float> a, const double2* __restrict__ r64,
                                              const SolverScal* outer) {
    const SysBlock q = sys_block(a);
    if (q.sys < 0) return;
    const double inv = 1.0 / outer->bnorm;
    double e[3] = {0.0, 0.0, 0.0};
    HZ_FOR_ELEMS(i, q.rw) {
        const double2 v = r64[i];
        const float2 r = mk<float>((float)(v.x * inv), (float)(v.y * inv));
        a.r[i] = r;
        const float2 w = a.rh[i];
        const double2 c = cdotacc(w.x, w.y, r.x, r.y, mk<double>(e[0], e[1]));
        e[0] = c.x;
        e[1] = c.y;
        e[2] = __builtin_fma((double)r.x, (double)r.x, e[2]);
        e[2] = __builtin_fma((double)r.y, (double)r.y, e[2]);
    }
    store_sys_partials<3>(a.part + kPartC * a.stride, a.stride, q.lb, e);
}

}  // namespace hz
