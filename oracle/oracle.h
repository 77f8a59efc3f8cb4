/*
 * CPU oracle interface -- TEST INFRASTRUCTURE ONLY (tests, smoke check and
 * the CPU-baseline leg of the benchmark).  Independent of the GPU library:
 * it includes none of its headers and the library includes none of these.
 */
#ifndef HELMZ_ORACLE_H
#define HELMZ_ORACLE_H
#include <stddef.h>

typedef struct { double re, im; } or_cplx_z; /* complex128 */
typedef struct { float re, im; } or_cplx_c;  /* complex64 */

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_BREAKDOWN = 2, OR_NONFINITE = 3, OR_INVALID = -1 };

typedef struct {
    int status;
    int iterations;       /* BiCGStab iterations (total inner ones for refinement) */
    int outer_steps;      /* refinement steps (0 for a plain solve) */
    int pad;
    double relres_recursive;
    double relres_true;
} or_info;

#define OR_DECLARE(P, C, R)                                                                          \
    void or_##P##spmv(int n, const int *row_ptr, const int *col_idx, const C *vals, const C *x, C *y); \
    C or_##P##dotc(int n, const C *x, const C *y);                                                    \
    R or_##P##nrm2(int n, const C *x);                                                                \
    void or_##P##axpy(int n, C alpha, const C *x, C *y);                                             \
    void or_##P##scal(int n, C alpha, C *x);                                                         \
    void or_##P##xmy(int n, const C *x, C *y);                                                       \
    size_t or_##P##bicgstab_work_elems(int n);                                                       \
    int or_##P##bicgstab(int n, const int *row_ptr, const int *col_idx, const C *vals, const C *b, C *x, \
                         double tol, int maxiter, int jacobi, int x0_zero, C *work, or_info *info);

OR_DECLARE(z, or_cplx_z, double)
OR_DECLARE(c, or_cplx_c, float)

/* refine.c (complex128 outer loop) */
int or_zbicgstab_mixed(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *vals, const or_cplx_z *b,
                       or_cplx_z *x, double tol, double inner_tol, int maxiter, int max_outer, int jacobi,
                       or_info *info);
void or_zcsr_conj_transpose(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *vals, int *t_row_ptr,
                            int *t_col_idx, or_cplx_z *t_vals);
void or_zgrad_vals(int n, const int *row_ptr, const int *col_idx, const or_cplx_z *lambda, const or_cplx_z *x,
                   or_cplx_z *grad_vals);

#endif
