/*
 * CPU oracle, complex128 drivers -- TEST INFRASTRUCTURE ONLY.
 *
 * Mixed-precision iterative refinement around the complex64 instantiation of
 * the BiCGStab oracle, and the two pieces of the adjoint (gradient) oracle.
 * Compiled with -O2 -ffp-contract=off; shares no code with the GPU library.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/*
 * Iterative refinement with a complex64 inner solver.  The paper's library
 * supports single precision as well as double (Section 1); this driver keeps
 * the residual, the correction update and the stopping test in complex128:
 *
 *   repeat: r = b - A x (FP64); stop when ||r|| / ||b|| <= tol;
 *           solve A d = r / ||r|| in complex64 (values of A rounded to
 *           complex64, BiCGStab to inner_tol, zero initial guess);
 *           x <- x + ||r|| d (FP64).
 *
 * x starts at zero.  info->iterations is the total of inner iterations and
 * info->outer_steps the number of corrections applied.
 */
int or_zbicgstab_mixed(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *vals, const or_cplx_z *b,
                       or_cplx_z *x, double tol, double inner_tol, int maxiter, int max_outer, int jacobi,
                       or_info *info)
{
    int nnz = row_ptr[n];
    memset(info, 0, sizeof(*info));
    or_cplx_c *v32 = malloc(sizeof(or_cplx_c) * (size_t)(nnz > 0 ? nnz : 1));
    or_cplx_c *r32 = malloc(sizeof(or_cplx_c) * (size_t)n);
    or_cplx_c *d32 = malloc(sizeof(or_cplx_c) * (size_t)n);
    or_cplx_c *w32 = malloc(sizeof(or_cplx_c) * or_cbicgstab_work_elems(n));
    or_cplx_z *r = malloc(sizeof(or_cplx_z) * (size_t)n);
    int status = OR_NOT_CONVERGED, outer = 0, inner_total = 0;
    double rel = 0;

    for (int p = 0; p < nnz; ++p) {
        v32[p].re = (float)vals[p].re;
        v32[p].im = (float)vals[p].im;
    }
    for (int i = 0; i < n; ++i)
        x[i].re = x[i].im = 0;
    double bn = or_znrm2(n, b);
    if (bn == 0) {
        status = OR_OK;
        goto done;
    }
    for (;;) {
        or_zspmv(n, row_ptr, col_idx, vals, x, r);
        for (int i = 0; i < n; ++i) {
            r[i].re = b[i].re - r[i].re;
            r[i].im = b[i].im - r[i].im;
        }
        double rn = or_znrm2(n, r);
        rel = rn / bn;
        if (!isfinite(rel)) { status = OR_NONFINITE; break; }
        if (rel <= tol) { status = OR_OK; break; }
        if (outer == max_outer) { status = OR_NOT_CONVERGED; break; }
        ++outer;
        for (int i = 0; i < n; ++i) {
            r32[i].re = (float)(r[i].re / rn);
            r32[i].im = (float)(r[i].im / rn);
        }
        or_info in;
        int st = or_cbicgstab(n, row_ptr, col_idx, v32, r32, d32, inner_tol, maxiter, jacobi, 1, w32, &in);
        inner_total += in.iterations;
        if (st == OR_INVALID) { status = OR_INVALID; break; }
        if (st == OR_NONFINITE) { status = OR_NONFINITE; break; }
        for (int i = 0; i < n; ++i) {
            x[i].re = x[i].re + rn * (double)d32[i].re;
            x[i].im = x[i].im + rn * (double)d32[i].im;
        }
    }
done:
    info->status = status;
    info->iterations = inner_total;
    info->outer_steps = outer;
    info->relres_recursive = rel;
    if (bn > 0) {
        or_zspmv(n, row_ptr, col_idx, vals, x, r);
        for (int i = 0; i < n; ++i) {
            r[i].re = b[i].re - r[i].re;
            r[i].im = b[i].im - r[i].im;
        }
        info->relres_true = or_znrm2(n, r) / bn;
    }
    free(v32); free(r32); free(d32); free(w32); free(r);
    return status;
}

/*
 * Conjugate transpose A^H of a CSR matrix, in CSR: entry (i, j, a) of A
 * becomes (j, i, conj(a)); within each output row, entries keep the order
 * of their source rows (ascending i), so columns come out sorted.
 */
void or_zcsr_conj_transpose(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *vals, int *t_row_ptr,
                            int *t_col_idx, or_cplx_z *t_vals)
{
    int nnz = row_ptr[n];
    for (int j = 0; j <= n; ++j)
        t_row_ptr[j] = 0;
    for (int p = 0; p < nnz; ++p)
        t_row_ptr[col_idx[p] + 1] += 1;
    for (int j = 0; j < n; ++j)
        t_row_ptr[j + 1] += t_row_ptr[j];
    int *fill = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; ++j)
        fill[j] = t_row_ptr[j];
    for (int i = 0; i < n; ++i)
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int q = fill[col_idx[p]]++;
            t_col_idx[q] = i;
            t_vals[q].re = vals[p].re;
            t_vals[q].im = -vals[p].im;
        }
    free(fill);
}

/*
 * Gradient of a real loss L(x), x = A^{-1} b, with respect to the stored
 * entries of A, in the real-pair convention g = dL/dRe + i dL/dIm.  With
 * lambda the solution of A^H lambda = dL/dx, a perturbation dA changes x by
 * -A^{-1} dA x, so dL = Re(sum_ij conj(-lambda_i conj(x_j)) dA_ij) and the
 * gradient of entry (i, j) is -lambda_i conj(x_j).
 */
void or_zgrad_vals(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *lambda, const or_cplx_z *x,
                   or_cplx_z *grad_vals)
{
    for (int i = 0; i < n; ++i)
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            or_cplx_z l = lambda[i], xc = x[col_idx[p]];
            /* -(l * conj(xc)) */
            grad_vals[p].re = -(l.re * xc.re + l.im * xc.im);
            grad_vals[p].im = -(l.im * xc.re - l.re * xc.im);
        }
}
