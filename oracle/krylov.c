/*
 * CPU oracle for the Helmholtz Krylov path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential complex arithmetic that the GPU library is checked
 * against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU library never does.  It shares no code with
 * the GPU kernels.
 *
 * This file is compiled twice: with OR_REAL=double / OR_PFX=z (complex128,
 * the paper's precision) and with OR_REAL=float / OR_PFX=c (complex64, used
 * only as the inner solver of the mixed-precision refinement).  Build flags:
 * -O2 -ffp-contract=off, so every product and sum below is rounded exactly
 * as written, in the order written.
 *
 * Complex numbers are pairs (re, im) with no padding, the memory layout of
 * the paper's complex structure (Section 4).
 *
 * A third build (OR_OMP, complex128 only, -fopenmp) exists only to time the
 * oracle on all host cores: it splits the row loop of the product and the
 * element-wise loops across threads, which changes no result, and lets
 * OpenMP sum the dot products and norms per thread, which changes their
 * rounding order.  Tests check the sequential build; the threaded one is
 * checked against it.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

#ifndef OR_REAL
#error "OR_REAL must be defined"
#endif
#define OR_CAT2(a, b) a##b
#define OR_CAT(a, b) OR_CAT2(a, b)
#define FN(name) OR_CAT(or_, OR_CAT(OR_PFX, name))
#define CPLX OR_CAT(or_cplx_, OR_PFX)

#include "oracle.h"

typedef OR_REAL real;

#ifdef OR_OMP
#define OR_PAR_FOR _Pragma("omp parallel for schedule(static)")
#define OR_PAR_SUM2 _Pragma("omp parallel for schedule(static) reduction(+ : ar, ai)")
#define OR_PAR_SUM1 _Pragma("omp parallel for schedule(static) reduction(+ : acc)")
#else
#define OR_PAR_FOR
#define OR_PAR_SUM2
#define OR_PAR_SUM1
#endif

/* ---- scalar complex arithmetic (textbook formulas, no FMA) ---- */
static CPLX cmk(real re, real im) { CPLX z; z.re = re; z.im = im; return z; }
static CPLX cadd(CPLX a, CPLX b) { return cmk(a.re + b.re, a.im + b.im); }
static CPLX csub(CPLX a, CPLX b) { return cmk(a.re - b.re, a.im - b.im); }
static CPLX cmul(CPLX a, CPLX b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
/* conj(a) * b */
static CPLX cmulc(CPLX a, CPLX b) { return cmk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }
static CPLX cdiv(CPLX a, CPLX b)
{
    real d = b.re * b.re + b.im * b.im;
    return cmk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
static int cfinite(CPLX a) { return isfinite(a.re) && isfinite(a.im); }
static int czero(CPLX a) { return a.re == 0 && a.im == 0; }

/*
 * Sparse matrix-vector product y = A x on CSR (Section 3.2; the paper's
 * 1-based IA/JA/AA become row_ptr/col_idx/vals, 0-based).  Row i sums its
 * entries in storage order.
 */
void FN(spmv)(int n, const int *row_ptr, const int *col_idx, const CPLX *vals, const CPLX *x, CPLX *y)
{
    OR_PAR_FOR
    for (int i = 0; i < n; ++i) {
        CPLX acc = cmk(0, 0);
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            acc = cadd(acc, cmul(vals[p], x[col_idx[p]]));
        y[i] = acc;
    }
}

/* Dot product (Section 5) with the first argument conjugated: sum conj(x_i) y_i. */
CPLX FN(dotc)(int n, const CPLX *x, const CPLX *y)
{
    real ar = 0, ai = 0;
    OR_PAR_SUM2
    for (int i = 0; i < n; ++i) {
        CPLX t = cmulc(x[i], y[i]);
        ar += t.re;
        ai += t.im;
    }
    return cmk(ar, ai);
}

/* Euclidean norm (Section 5, NormL2): sqrt(sum re^2 + im^2). */
real FN(nrm2)(int n, const CPLX *x)
{
    real acc = 0;
    OR_PAR_SUM1
    for (int i = 0; i < n; ++i)
        acc += x[i].re * x[i].re + x[i].im * x[i].im;
    return sqrt(acc);
}

/* y <- alpha x + y (Section 5, the complex axpy). */
void FN(axpy)(int n, CPLX alpha, const CPLX *x, CPLX *y)
{
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        y[i] = cadd(cmul(alpha, x[i]), y[i]);
}

/* y <- alpha x (Section 5, scale). */
void FN(scal)(int n, CPLX alpha, CPLX *x)
{
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        x[i] = cmul(alpha, x[i]);
}

/* y_i <- x_i * y_i (Section 5, element-wise product). */
void FN(xmy)(int n, const CPLX *x, CPLX *y)
{
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        y[i] = cmul(x[i], y[i]);
}

/* z <- M^{-1} w for the Jacobi preconditioner M = diag(A), or a copy. */
static void apply_prec(int n, const CPLX *dinv, const CPLX *w, CPLX *z)
{
    if (!dinv) {
        memcpy(z, w, sizeof(CPLX) * (size_t)n);
        return;
    }
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        z[i] = cmul(dinv[i], w[i]);
}

size_t FN(bicgstab_work_elems)(int n) { return (size_t)9 * (size_t)n; }

/*
 * Preconditioned BiCGStab (Section 7: the P-BiCGSTAB the paper runs, the
 * bi-conjugate gradient stabilised method of the Saad textbook it cites),
 * right-preconditioned by M = I or M = diag(A).  Inner products are the
 * conjugated dot product above.  Scalars rho, alpha, omega start at 1, the
 * shadow residual is the initial residual, and convergence is tested on the
 * recursively updated residual relative to ||b||, both after the half step
 * (||s||) and after the full step (||r||).  A half-step exit counts as a
 * full iteration.  Breakdown is an exact zero of rho, <rhat, v>, <t, t> or
 * omega; a non-finite scalar stops with OR_NONFINITE.
 *
 * work must hold FN(bicgstab_work_elems)(n) complex entries.
 */
int FN(bicgstab)(int n, const int *row_ptr, const int *col_idx, const CPLX *vals, const CPLX *b, CPLX *x,
                 double tol, int maxiter, int jacobi, int x0_zero, CPLX *work, or_info *info)
{
    CPLX *r = work, *rhat = work + n, *p = work + 2 * (size_t)n, *v = work + 3 * (size_t)n;
    CPLX *s = work + 4 * (size_t)n, *t = work + 5 * (size_t)n, *phat = work + 6 * (size_t)n;
    CPLX *shat = work + 7 * (size_t)n, *dinv = NULL;
    int status = OR_NOT_CONVERGED, it = 0;
    double resid = 0;

    memset(info, 0, sizeof(*info));
    if (jacobi) {
        dinv = work + 8 * (size_t)n;
        for (int i = 0; i < n; ++i) {
            CPLX d = cmk(0, 0);
            for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
                if (col_idx[q] == i)
                    d = vals[q];
            if (czero(d))
                return info->status = OR_INVALID;
            dinv[i] = cdiv(cmk(1, 0), d);
        }
    }
    if (x0_zero)
        for (int i = 0; i < n; ++i)
            x[i] = cmk(0, 0);

    real bn = FN(nrm2)(n, b);
    if (bn == 0) {
        for (int i = 0; i < n; ++i)
            x[i] = cmk(0, 0);
        info->status = OR_OK;
        return OR_OK;
    }
    /* r = b - A x ; rhat = r */
    FN(spmv)(n, row_ptr, col_idx, vals, x, r);
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        r[i] = csub(b[i], r[i]);
    memcpy(rhat, r, sizeof(CPLX) * (size_t)n);
    CPLX rho_prev = cmk(1, 0), alpha = cmk(1, 0), omega = cmk(1, 0);
    for (int i = 0; i < n; ++i)
        v[i] = p[i] = cmk(0, 0);
    resid = FN(nrm2)(n, r) / bn;
    if (resid <= tol) {
        info->status = OR_OK;
        info->relres_recursive = resid;
        return OR_OK;
    }

    for (it = 1; it <= maxiter; ++it) {
        CPLX rho = FN(dotc)(n, rhat, r);
        if (!cfinite(rho)) { status = OR_NONFINITE; break; }
        if (czero(rho)) { status = OR_BREAKDOWN; break; }
        if (it == 1) {
            memcpy(p, r, sizeof(CPLX) * (size_t)n);
        } else {
            CPLX beta = cmul(cdiv(rho, rho_prev), cdiv(alpha, omega));
            if (!cfinite(beta)) { status = OR_NONFINITE; break; }
            OR_PAR_FOR
            for (int i = 0; i < n; ++i)
                p[i] = cadd(r[i], cmul(beta, csub(p[i], cmul(omega, v[i]))));
        }
        apply_prec(n, dinv, p, phat);
        FN(spmv)(n, row_ptr, col_idx, vals, phat, v);
        CPLX sigma = FN(dotc)(n, rhat, v);
        if (!cfinite(sigma)) { status = OR_NONFINITE; break; }
        if (czero(sigma)) { status = OR_BREAKDOWN; break; }
        alpha = cdiv(rho, sigma);
        OR_PAR_FOR
        for (int i = 0; i < n; ++i)
            s[i] = csub(r[i], cmul(alpha, v[i]));
        resid = FN(nrm2)(n, s) / bn;
        if (!isfinite(resid)) { status = OR_NONFINITE; break; }
        if (resid <= tol) {
            OR_PAR_FOR
            for (int i = 0; i < n; ++i)
                x[i] = cadd(x[i], cmul(alpha, phat[i]));
            status = OR_OK;
            break;
        }
        apply_prec(n, dinv, s, shat);
        FN(spmv)(n, row_ptr, col_idx, vals, shat, t);
        CPLX tt = FN(dotc)(n, t, t);
        if (!cfinite(tt)) { status = OR_NONFINITE; break; }
        if (czero(tt)) { status = OR_BREAKDOWN; break; }
        omega = cdiv(FN(dotc)(n, t, s), tt);
        if (!cfinite(omega)) { status = OR_NONFINITE; break; }
        OR_PAR_FOR
        for (int i = 0; i < n; ++i) {
            x[i] = cadd(cadd(x[i], cmul(alpha, phat[i])), cmul(omega, shat[i]));
            r[i] = csub(s[i], cmul(omega, t[i]));
        }
        resid = FN(nrm2)(n, r) / bn;
        if (!isfinite(resid)) { status = OR_NONFINITE; break; }
        if (resid <= tol) { status = OR_OK; break; }
        if (czero(omega)) { status = OR_BREAKDOWN; break; }
        rho_prev = rho;
    }
    if (it > maxiter)
        it = maxiter;
    info->status = status;
    info->iterations = it;
    info->relres_recursive = resid;
    /* true residual ||b - A x|| / ||b|| in this instantiation's precision */
    FN(spmv)(n, row_ptr, col_idx, vals, x, t);
    OR_PAR_FOR
    for (int i = 0; i < n; ++i)
        t[i] = csub(b[i], t[i]);
    info->relres_true = FN(nrm2)(n, t) / bn;
    return status;
}
