/*
 * helmz -- complex-double Krylov solves of sparse Helmholtz systems on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Cheik Ahamed & Magoules, "Accelerated solution
 * of Helmholtz equation with Iterative Krylov Methods on GPU": complex
 * sparse matrix-vector product on CSR storage (Sections 3.2 and 6), the
 * complex BLAS-1 operations dot product, norm and axpy (Section 5), and the
 * preconditioned BiCGStab solve of A x = b with zero initial guess, a
 * residual tolerance and an iteration limit (Section 7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex numbers are (re, im) pairs with no padding: the paper's complex
 *    structure (Section 4), the same layout as torch.complex128 /
 *    torch.complex64.  hz_c128 arrays must be 16-byte aligned, hz_c64 arrays
 *    8-byte aligned.
 *  - CSR is 0-based: row i occupies [row_ptr[i], row_ptr[i+1]) of col_idx
 *    and vals (the paper's 1-based IA/JA/AA).  row_ptr has n+1 int32
 *    entries with row_ptr[0] = 0 and row_ptr[n] = nnz; 0 <= col_idx < n.
 *    Unless HZ_VALIDATE is passed, malformed CSR is undefined behaviour.
 *  - Every array pointer is a DEVICE pointer owned by the caller.  The
 *    library never frees or retains them.  Work is enqueued on `stream`
 *    (a hipStream_t; NULL means the default stream).
 *  - Return value: HZ_OK (0), a positive solver status, or a negative error.
 *    No call aborts or throws.  hz_strerror() names every code.
 *  - A handle holds per-device scratch (reduction partials, device scalars,
 *    pinned host words); calls that share a handle must be issued from one
 *    host thread at a time.  A handle is bound to the device that was
 *    current when it was created.
 */
#ifndef HELMZ_H
#define HELMZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hz_c128;
typedef struct { float re, im; } hz_c64;
typedef struct hz_handle hz_handle;
typedef void *hz_stream; /* hipStream_t */

/* status and error codes */
enum {
    HZ_OK = 0,
    HZ_NOT_CONVERGED = 1, /* maxiter reached; x holds the last iterate      */
    HZ_BREAKDOWN = 2,     /* rho, <rhat,v>, <t,t> or omega became exactly 0 */
    HZ_NONFINITE = 3,     /* a NaN/Inf scalar appeared                      */
    HZ_ERR_INVALID = -1,  /* bad argument or malformed CSR (validated)      */
    HZ_ERR_HIP = -2,      /* a HIP runtime call failed                      */
    HZ_ERR_WORKSPACE = -3, /* workspace missing, misaligned or too small    */
    HZ_ERR_TOO_LARGE = -4  /* beyond the static scratch (noalloc solve)     */
};

/* solver flags (bitwise or) */
#define HZ_PRECOND_NONE 0x0
#define HZ_PRECOND_JACOBI 0x1 /* right preconditioner M = diag(A)          */
#define HZ_X0_ZERO 0x4        /* ignore x on entry, start from 0 (paper)   */
#define HZ_VALIDATE 0x8       /* check CSR structure on the device first   */
#define HZ_SYMMETRIC 0x10     /* caller asserts A = A^T (adjoint shortcut) */
#define HZ_REORDER 0x20       /* always renumber by level sets first       */
#define HZ_NO_REORDER 0x40    /* never renumber (smaller workspace)        */
#define HZ_RELIABLE 0x80      /* mixed: reliable updates, not restarts     */

typedef struct {
    int status;              /* HZ_OK / HZ_NOT_CONVERGED / HZ_BREAKDOWN / HZ_NONFINITE */
    int iterations;          /* iterations: BiCGStab's (inner total for mixed),
                                BiCGstab(l)'s cycles, TFQMR's full iterations */
    int outer_steps;         /* refinement corrections (mixed only)         */
    int renumbered;          /* 1 if solved in the level-set numbering      */
    double relres_recursive; /* last ||r||/||b|| of the recursive residual  */
    double relres_true;      /* ||b - A x|| / ||b||, recomputed in FP64     */
    int breakdown;           /* status HZ_BREAKDOWN: which scalar was 0     */
    int reserved;
} hz_solve_info;

/* hz_solve_info.breakdown: the quantity that became exactly zero */
enum {
    HZ_BD_NONE = 0,
    HZ_BD_RHO = 1,    /* rho = <rhat, r>                                  */
    HZ_BD_RHAT_V = 2, /* <rhat, v>, the denominator of alpha              */
    HZ_BD_TT = 3,     /* <t, t>, the denominator of omega                 */
    HZ_BD_OMEGA = 4,  /* omega itself                                     */
    HZ_BD_MR = 5      /* BiCGstab(l): the minimal-residual system is singular */
};

/* Handle with scratch for the standalone reductions and the solvers, the
 * autotuned launch shapes, and a cache of up to 32 instantiated HIP graphs of
 * solver iteration chunks with the stream they are captured on.  A chunk of
 * iterations with the same kernels and arguments as a cached one (same
 * matrix, vectors and workspace) is replayed with one hipGraphLaunch on the
 * caller's stream; results are bitwise those of direct launches, which the
 * environment variable HZ_NO_GRAPH=1 selects.  Allocates device memory and
 * the capture stream once, and arms the slots of zdotc / dznrm2 with a kernel
 * on the null stream that it waits for, so it must not be called while a
 * stream of the device is being captured; returns HZ_ERR_HIP if any of this
 * fails.  One handle per device, used by one host thread at a time. */
int hz_handle_create(hz_handle **handle);
int hz_handle_destroy(hz_handle *handle);

/* Text for any return code of this library (never NULL). */
const char *hz_strerror(int code);

/*
 * y = A x, complex128 CSR sparse matrix-vector product (Sections 3.2, 6).
 * x and y hold n entries and must not overlap.  n = 0 is a no-op.
 * Runs in one of two forms (HZ_SPMV_FORM_*; see hz_autotune_spmv): vector
 * rows, L lanes per row, with the next rows' loads issued while the current
 * rows' x gathers are in flight; or block tiles of 64 rows whose entries the
 * whole block loads contiguously and multiplies into LDS before each row is
 * summed there.  The result is bitwise reproducible for a given form and L.
 */
int csr_zspmv(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
              const hz_c128 *vals, const hz_c128 *x, hz_c128 *y);

enum { HZ_SPMV_FORM_ROWS = 0, HZ_SPMV_FORM_TILES = 1 };

/*
 * Autotuner of the launch shapes for one matrix.  Two choices are made:
 *  - the lanes per row L (2 ... 64, so 64/L rows per wavefront, or 1 for
 *    the block-tile row loop) of the solver kernels' fused row products,
 *    timed on that row product;
 *  - the form of the standalone product (csr_zspmv, csr_cspmv,
 *    csr_zspmv_rect): vector rows with each L, or block tiles.
 * Each candidate is timed on the caller's matrix and vectors (two rounds of
 * 5 launches after 2 warm-up launches, HIP events on `stream`); the fastest
 * (the untuned choice unless another is more than 3 % faster) are
 * recorded in the handle for this (row_ptr, col_idx, n, nnz), and later
 * products and solves on the same handle with the same index arrays use
 * them (results change only by summation order).  Without tuning, the
 * solver kernels use vector rows with the smallest power of two L not below
 * half the mean row length (block tiles for a one-system FP64 solve whose
 * values exceed 128 MiB), and the standalone product uses block tiles when
 * the mean row length is at most 16 entries, else vector rows with that L.  Writes the solver lane count to *lanes, and, where the pointers
 * are not NULL, the standalone form to *form (HZ_SPMV_FORM_*) and its lane
 * count to *form_lanes (host memory).  y is overwritten with A x.
 * Synchronises the stream.  The environment variables HZ_SPMV_LANES (a lane
 * count) and HZ_SPMV_FORM ("rows" or "tiles"), when set, override the rule
 * and the tuned choices.
 */
int hz_autotune_spmv(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                     const hz_c128 *vals, const hz_c128 *x, hz_c128 *y, int *lanes, int *form, int *form_lanes);

/*
 * Records launch shapes for one matrix without timing them, as if
 * hz_autotune_spmv had chosen them (a tuning cache kept across processes
 * calls this with the choice it stored for a matrix of the same shape):
 * lanes is the solver kernels' lane count (1 for the block-tile row loop,
 * or 2 ... 64), form HZ_SPMV_FORM_ROWS with form_lanes 2 ... 64, or
 * HZ_SPMV_FORM_TILES with form_lanes 4.  Host-only; returns HZ_ERR_INVALID
 * for other values.
 */
int hz_autotune_set(hz_handle *handle, int n, int nnz, const int *row_ptr, const int *col_idx, int lanes, int form,
                    int form_lanes);

/* Same product with complex64 values, vectors and arithmetic. */
int csr_cspmv(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
              const hz_c64 *vals, const hz_c64 *x, hz_c64 *y);

/*
 * *out = sum_i conj(x_i) y_i (Section 5, dot product; the first argument is
 * conjugated).  out is a device pointer; nothing is synchronised.  One
 * launch: each block publishes its total in a slot of the handle (an
 * agent-scope atomic store), the grid's last block waits for every slot and
 * adds the totals in index order, so the sum order is fixed for a given n
 * and repeated calls are bitwise identical.  The wait is bounded (2 s of the
 * device clock, or HZ_B1_WAIT_TICKS ticks read at hz_handle_create; 0 gives
 * up at once): a wait that gives up writes NaN and leaves the handle's
 * reductions broken, every later zdotc and dznrm2 on it writing NaN, until
 * the handle is destroyed.  zdotc and dznrm2 share the handle's slots and
 * hz_stream_read its partials: calls on one handle must not overlap in time
 * (one stream, or serialised streams).
 */
int zdotc(hz_handle *handle, hz_stream stream, int n, const hz_c128 *x, const hz_c128 *y, hz_c128 *out);

/* *out = ||x||_2 = sqrt(sum |x_i|^2) (Section 5, norm), device pointer;
 * one launch, slots and bounded wait as for zdotc. */
int dznrm2(hz_handle *handle, hz_stream stream, int n, const hz_c128 *x, double *out);

/* y <- alpha x + y (Section 5, complex axpy); alpha by value; x may equal
 * y, other overlaps are invalid.  One streaming pass, four 16-byte loads of
 * each vector in flight per thread. */
int zaxpy(hz_handle *handle, hz_stream stream, int n, hz_c128 alpha, const hz_c128 *x, hz_c128 *y);

/* Device workspace (bytes) that zbicgstab_solve needs for this n, nnz,
 * flags.  Unless HZ_NO_REORDER is passed it includes room for a renumbered
 * copy of the matrix (20 nnz + 80 n bytes and sort scratch). */
size_t zbicgstab_workspace_bytes(int n, int nnz, int flags);

/*
 * Solve A x = b by preconditioned BiCGStab (Section 7: the paper's
 * P-BiCGSTAB), complex128.  Right preconditioner M = I or M = diag(A)
 * (HZ_PRECOND_JACOBI).  The shadow residual is the initial residual;
 * convergence is ||r|| / ||b|| <= rtol on the recursive residual, tested
 * after the half step (s) and after the full step (r).  x is in/out: the
 * initial guess on entry (zero if HZ_X0_ZERO), the solution on return.
 * ws is a device buffer of at least zbicgstab_workspace_bytes(n, nnz,
 * flags) bytes, 256-byte aligned, owned by the caller.  The call
 * synchronises `stream` and fills *info (host memory).  Returns the solver
 * status (also in info->status) or a negative error.
 *
 * Renumbering (not in the paper; a locality step of this library): with
 * HZ_REORDER, or by default when more than 5 % of the entries lie more than
 * 32,768 rows from the diagonal, the solve runs on P A P^T (P x) = P b for
 * the level-set permutation P of csr_level_order and scatters x back.
 * BiCGStab with Jacobi scaling is invariant under a symmetric permutation,
 * so this changes only the rounding order.  HZ_NO_REORDER forbids it;
 * passing both flags is HZ_ERR_INVALID.  Batched solves never renumber.
 */
int zbicgstab_solve(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                    const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol, int maxiter, int flags, void *ws,
                    size_t ws_bytes, hz_solve_info *info);

/*
 * zbicgstab_solve_async: the same solve with nothing on the host waiting for
 * the stream (Section 7's iteration control kept on the device): every
 * launch of up to maxiter iterations is enqueued in chunks of 64 (kernels
 * after the exit return at entry, a few microseconds each, so maxiter should
 * be near the expected count), and the result is written by a kernel to
 * info_dev, a device hz_solve_info (8-byte aligned), when the stream reaches
 * it.  b, x, ws and info_dev must stay valid until then.  One system, FP64,
 * caller's numbering: HZ_REORDER, HZ_VALIDATE and HZ_RELIABLE are invalid,
 * renumbering never happens (workspace as for zbicgstab_solve with
 * HZ_NO_REORDER).  The launch map is written into ws by a kernel, so the
 * call allocates nothing and never waits; iteration graphs cached by the
 * handle are evicted only after their last launch has completed.  A zero
 * diagonal under Jacobi is reported as info_dev->status =
 * HZ_ERR_INVALID.  Returns HZ_OK once enqueued, or an argument error.
 */
int zbicgstab_solve_async(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                          const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol, int maxiter, int flags,
                          void *ws, size_t ws_bytes, hz_solve_info *info_dev);

/*
 * zbicgstab_solve_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The solve of zbicgstab_solve_async (same kernels, same
 * arguments and flags, same device-side info_dev) with no workspace
 * argument: its workspace is a static device array of
 * zbicgstab_noalloc_max_bytes() bytes (96 MiB) in the library, one per GPU,
 * held until the process ends.  The call allocates nothing, records no
 * memset and captures no graph (its iterations are launched directly), and
 * never waits on the host.  Systems whose workspace (zbicgstab_workspace_bytes
 * with HZ_NO_REORDER) exceeds the array return HZ_ERR_TOO_LARGE: that is
 * about 780,000 rows with no preconditioner (128 bytes per row), or about
 * 260,000 rows of 15 entries under Jacobi (the 210k-row cylinder fits).
 * Every call on one GPU uses the same array
 * and initialises all of it that it reads, so results do not depend on
 * earlier calls; calls that overlap in time on one GPU (other streams, or
 * other threads) race on it and must be serialised by the caller.
 */
size_t zbicgstab_noalloc_max_bytes(void);
int zbicgstab_solve_noalloc(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr,
                            const int *col_idx, const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol,
                            int maxiter, int flags, hz_solve_info *info_dev);

/*
 * BiCGstab(l), the paper's P-BiCGSTAB(l) (Section 7, iterative Krylov
 * methods; l = 8 in its speed-up tables), in Sleijpen and Fokkema's form:
 * each cycle makes l Bi-CG steps, then takes the coefficients that minimise
 * ||r_0 - sum_j gamma_j r_j||_2 over its residual basis r_1 .. r_l (normal
 * equations of the basis' Gram matrix, scaled to unit diagonal, solved by
 * Cholesky on the device).  Arguments, flags, workspace and return codes as
 * for zbicgstab_solve, with 1 <= ell <= 8 and maxcycles the limit on cycles
 * (each cycle is l Bi-CG steps and 2 l products).  The relative recursive
 * residual is tested at the end of every cycle.  info->iterations counts
 * cycles; a breakdown is an exact zero rho (HZ_BD_RHO), <r~, A u_j>
 * (HZ_BD_RHAT_V), omega = gamma_l (HZ_BD_OMEGA), or a minimal-residual system
 * that is not positive definite in floating point (HZ_BD_MR).  HZ_RELIABLE
 * is invalid here.
 */
size_t zbicgstabl_workspace_bytes(int n, int nnz, int ell, int flags);
int zbicgstabl_solve(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                     const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, int ell, double rtol, int maxcycles,
                     int flags, void *ws, size_t ws_bytes, hz_solve_info *info);

/*
 * TFQMR, the paper's P-TFQMR (Section 7, iterative Krylov methods): Freund's
 * transpose-free QMR in the form of Saad's book, two products per iteration,
 * right Jacobi preconditioning as for zbicgstab_solve.  The stopping test is
 * the quasi-residual bound sqrt(m + 2) tau_{m+1} <= rtol ||b|| after every
 * half step m, which bounds the true relative residual (reported in
 * info->relres_true); info->relres_recursive is the bound, info->iterations
 * counts full iterations (an exit after the first half step counts the
 * iteration).  Arguments, flags, workspace and return codes as for
 * zbicgstab_solve; a breakdown is an exact zero <r~, v> (HZ_BD_RHAT_V) or rho
 * (HZ_BD_RHO).  HZ_RELIABLE is invalid here.
 */
size_t ztfqmr_workspace_bytes(int n, int nnz, int flags);
int ztfqmr_solve(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                 const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol, int maxiter, int flags, void *ws,
                 size_t ws_bytes, hz_solve_info *info);

/*
 * Storage formats beside CSR (Section 3.2 names coordinate, ELLPACK and
 * hybrid storage as the alternatives to its CSR; SELL-C-sigma is Kreutzer et
 * al.'s sliced ELLPACK).  All arrays are device memory owned by the caller,
 * indices 0-based int32, values interleaved complex128.  Conversions are
 * set-up calls: they validate the CSR arrays (HZ_ERR_INVALID), synchronise the
 * stream and may be slow; the products are ordinary stream-ordered launches
 * that trust the arrays the conversions wrote.
 *
 * ELL of width K: entry k of row i at k*n + i (column-major), padding column
 * -1 and value 0.  HYB of width K: that ELL part holding the first
 * min(len_i, K) entries of each row, plus the rest as COO triplets (row,
 * column, value) in CSR order.  SELL-C-sigma with t lanes per row: rows
 * sorted by decreasing length within windows of sigma rows (ties keep row
 * order; sigma = 1 keeps CSR order), sorted position p holding row perm[p];
 * chunk c = p / C, row r = p % C; chunk width w_c = its longest row rounded
 * up to a multiple of t, chunk_ptr[c + 1] - chunk_ptr[c] = C w_c, entry k at
 * chunk_ptr[c] + (k / t) C t + r t + k % t; padding column -1, value 0, the
 * last chunk padded with empty rows.  t = 1 is Kreutzer et al.'s layout,
 * t > 1 gives each row t neighbouring slots (Anzt et al.'s SELL-P).
 *
 * csr_format_workspace_bytes: scratch for csr_row_stats, csr_to_hyb and
 * csr_sell_analyze on n rows (256-byte aligned).
 * csr_row_stats: the longest row and the default HYB width (the largest K
 * that at least ceil(n/3) rows reach: Bell and Garland's rule).
 * csr_to_hyb: writes ELL(K) (K*n slots; K = the longest row gives plain ELL)
 * and the COO remainder; *coo_nnz receives the remainder's size, and if it
 * exceeds coo_cap nothing is written and HZ_ERR_WORKSPACE is returned (call
 * with coo_cap = 0 to query).
 * hyb_zspmv: y = A x from ELL(K) + COO (coo_nnz may be 0); x, y of n entries,
 * no overlap.  Row sums: the ELL slots in order, plus the COO entries'.
 * csr_sell_analyze: perm (n entries) and chunk_ptr (ceil(n/C) + 1 entries);
 * *slots receives chunk_ptr's last entry, the length of the value and
 * column arrays.  1 <= C <= 1024, t in {1, 2, 4, 8}, sigma = 1 or a
 * multiple of C.
 * csr_to_sell: fills sell_col / sell_val (slots entries) from CSR, perm and
 * chunk_ptr; HZ_ERR_INVALID if they do not fit the matrix or slots.  C and t
 * must be those of the csr_sell_analyze call that wrote perm and chunk_ptr
 * (chunk_ptr is read at ceil(n/C) + 1 entries).
 * sell_zspmv: y = A x; y[perm[p]] receives sorted row p's sum (C and t as
 * for csr_to_sell).
 */
size_t csr_format_workspace_bytes(int n);
int csr_row_stats(hz_handle *handle, hz_stream stream, int n, const int *row_ptr, void *ws, size_t ws_bytes,
                  int *max_len, int *hyb_width);
int csr_to_hyb(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
               const hz_c128 *vals, int K, int *ell_col, hz_c128 *ell_val, int coo_cap, int *coo_row, int *coo_col,
               hz_c128 *coo_val, void *ws, size_t ws_bytes, int *coo_nnz);
int hyb_zspmv(hz_handle *handle, hz_stream stream, int n, int K, const int *ell_col, const hz_c128 *ell_val,
              int coo_nnz, const int *coo_row, const int *coo_col, const hz_c128 *coo_val, const hz_c128 *x,
              hz_c128 *y);
int csr_sell_analyze(hz_handle *handle, hz_stream stream, int n, const int *row_ptr, int C, int sigma, int t,
                     int *perm, int64_t *chunk_ptr, void *ws, size_t ws_bytes, int64_t *slots);
int csr_to_sell(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                const hz_c128 *vals, int C, int t, const int *perm, const int64_t *chunk_ptr, int64_t slots,
                int *sell_col, hz_c128 *sell_val);
int sell_zspmv(hz_handle *handle, hz_stream stream, int n, int C, int t, const int *perm, const int64_t *chunk_ptr,
               const int *sell_col, const hz_c128 *sell_val, const hz_c128 *x, hz_c128 *y);

/*
 * Workspace (bytes) for zbicgstab_solve_varbatch.  row_off is a HOST array of
 * nsys+1 row offsets (row_off[0] = 0, non-decreasing).
 */
size_t zbicgstab_varbatch_workspace_bytes(int nsys, const int *row_off, int nnz, int flags);

/*
 * Solve nsys independent systems A_j x_j = b_j of uneven sizes in one launch
 * sequence (batching is an extension of Section 7's solve): the systems are
 * the diagonal blocks of one block-diagonal CSR matrix (rows row_off[j] ..
 * row_off[j+1]-1 of row_ptr/col_idx/vals, GLOBAL column indices inside the
 * block), b and x are the concatenated vectors.  Every system runs its own
 * preconditioned BiCGStab with its own scalars, convergence test and exit,
 * exactly as zbicgstab_solve would; systems that finish early stop consuming
 * bandwidth.  infos is a HOST array of nsys results.  Returns the largest
 * status over the systems, or a negative error.  Flags, stream and
 * workspace as for zbicgstab_solve; systems are never renumbered.
 */
int zbicgstab_solve_varbatch(hz_handle *handle, hz_stream stream, int nsys, const int *row_off, int nnz,
                             const int *row_ptr, const int *col_idx, const hz_c128 *vals, const hz_c128 *b,
                             hz_c128 *x, double rtol, int maxiter, int flags, void *ws, size_t ws_bytes,
                             hz_solve_info *infos);

/* Workspace (bytes) for zbicgstab_solve_batched: nsys systems of n rows. */
size_t zbicgstab_batched_workspace_bytes(int nsys, int n, int nnz, int flags);

/*
 * Solve nsys systems A_j x_j = b_j that share one sparsity pattern (a
 * frequency sweep K - k_j^2 M + i k_j B on one mesh); batching is an
 * extension of Section 7's solve.  Up to 16 systems run in one launch
 * sequence; more run as near-equal groups of up to 16, one group after
 * another, in order of a diagonal key (the sum of Re A_j(i,i) over up to
 * 1,024 evenly spaced rows; ties by index), so that in a sweep a group holds
 * neighbouring wavenumbers with similar iteration counts.  1 <= nsys <= 256 and
 * n * nsys < 2^31.  Layout is system-minor: vals[p * nsys + j] is entry p
 * of system j (nnz * nsys values), b[i * nsys + j] and x[i * nsys + j]
 * element i of system j.  Every system runs its own preconditioned BiCGStab
 * (HZ_PRECOND_JACOBI scales each system by its own diagonal) with its own
 * scalars, convergence test and exit; a system's arithmetic does not depend
 * on the others, so permuting the systems permutes the results bitwise.
 * row_ptr/col_idx are read once per row for all systems.  infos is a HOST
 * array of nsys results; returns the largest status or a negative error.
 * Flags (HZ_X0_ZERO, HZ_VALIDATE, HZ_PRECOND_JACOBI), stream and workspace
 * as for zbicgstab_solve; systems are never renumbered.
 */
int zbicgstab_solve_batched(hz_handle *handle, hz_stream stream, int nsys, int n, int nnz, const int *row_ptr,
                            const int *col_idx, const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol,
                            int maxiter, int flags, void *ws, size_t ws_bytes, hz_solve_info *infos);

/* Workspace (bytes) for zbicgstab_solve_sweep: nsys wavenumbers on n rows. */
size_t zbicgstab_sweep_workspace_bytes(int nsys, int n, int nnz, int flags);

/*
 * Frequency sweep: solve A(k_j) x_j = b_j for nsys wavenumbers k_j with
 * A(k) = K - k^2 M + i k B, the finite-element Helmholtz operator (stiffness,
 * mass and boundary matrices of Section 2's equation) on one pattern.  K, M
 * and B are real DEVICE arrays of nnz doubles on row_ptr/col_idx (8-byte
 * aligned); ks is a HOST array of nsys finite wavenumbers.  The same
 * per-system BiCGStab as zbicgstab_solve_batched (same limits, flags,
 * layout of b and x [n][nsys], infos and return value), but the entries of
 * every system are formed on the fly from the three shared arrays: 24 bytes
 * per entry for the whole sweep instead of 16 bytes per entry per system.
 * Under HZ_PRECOND_JACOBI each system is scaled by its own diagonal
 * K_ii - k_j^2 M_ii + i k_j B_ii, applied to the gathered vectors.
 */
int zbicgstab_solve_sweep(hz_handle *handle, hz_stream stream, int nsys, int n, int nnz, const int *row_ptr,
                          const int *col_idx, const double *K, const double *M, const double *B, const double *ks,
                          const hz_c128 *b, hz_c128 *x, double rtol, int maxiter, int flags, void *ws,
                          size_t ws_bytes, hz_solve_info *infos);

/* Device workspace (bytes) that zbicgstab_solve_mixed needs. */
size_t zbicgstab_mixed_workspace_bytes(int n, int nnz, int flags);

/*
 * Solve A x = b to ||b - A x|| / ||b|| <= rtol by iterative refinement with
 * a complex64 inner BiCGStab.  The paper's library provides single as well
 * as double precision (Section 1); this entry point combines them: the
 * residual r = b - A x, the correction x <- x + ||r|| d, the norms and the
 * stopping test are complex128, while each correction solves A d = r/||r||
 * to inner_rtol with the values of A (column-scaled by D^{-1} under
 * HZ_PRECOND_JACOBI) rounded to complex64 and complex64 vectors and SpMV
 * (Krylov scalars and reductions in FP64).  At most max_outer corrections,
 * each of at most maxiter inner iterations.  info->iterations is the total
 * of inner iterations, info->outer_steps the number of corrections, and
 * info->relres_true the final FP64 residual.  Workspace, stream, x,
 * renumbering and status conventions as for zbicgstab_solve.
 *
 * With HZ_RELIABLE the corrections are not separate solves: one complex64
 * BiCGStab runs on A D^{-1} y = b / ||b|| and, whenever its recursive
 * residual has fallen by the factor inner_rtol (0 < inner_rtol < 1, e.g.
 * 0.1) since the last update or the iteration has ended, a reliable update
 * (Sleijpen and van der Vorst) moves ||b|| D^{-1} y into the FP64 x, forms
 * r = b - A x in FP64 and replaces the complex64 residual by r / ||b||,
 * keeping the Krylov directions.  The decision is on the FP64 residual;
 * info->outer_steps counts the updates (at most max_outer) and
 * info->iterations the complex64 iterations (at most maxiter in total).
 */
int zbicgstab_solve_mixed(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr,
                          const int *col_idx, const hz_c128 *vals, const hz_c128 *b, hz_c128 *x, double rtol,
                          double inner_rtol, int maxiter, int max_outer, int flags, void *ws, size_t ws_bytes,
                          hz_solve_info *info);

/*
 * y = A x for a rectangular m x ncols complex128 CSR matrix (same storage
 * as csr_zspmv; row_ptr has m+1 entries, 0 <= col_idx < ncols).  Used to
 * chain entry gradients to the parameters the entries depend on.
 */
int csr_zspmv_rect(hz_handle *handle, hz_stream stream, int m, int ncols, int nnz, const int *row_ptr,
                   const int *col_idx, const hz_c128 *vals, const hz_c128 *x, hz_c128 *y);

/*
 * grad_vals[p] = -lambda_i * conj(x_j) for every stored entry p = (i, j):
 * the gradient of a real loss L with respect to the entries of A, where x
 * solves A x = b and lambda solves A^H lambda = dL/dx (real-pair convention
 * g = dL/dRe + i dL/dIm, as torch uses).  Differentiation of the paper's
 * solve (Section 7) is an extension; the formula follows from
 * dx = -A^{-1} dA x.
 */
int csr_zgrad_vals(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                   const hz_c128 *lambda, const hz_c128 *x, hz_c128 *grad_vals);

/* Device workspace (bytes) that zbicgstab_adjoint needs for these flags. */
size_t zbicgstab_adjoint_workspace_bytes(int n, int nnz, int flags);

/*
 * Backward of x = A^{-1} b (Section 7's solve, differentiated): given
 * grad_x = dL/dx (real-pair convention), solve A^H lambda = grad_x by the
 * same preconditioned BiCGStab (rtol, maxiter, HZ_PRECOND_JACOBI as for
 * zbicgstab_solve; the initial guess is zero), write grad_b = lambda and,
 * if grad_vals is not NULL, grad_vals[p] = -lambda_i conj(x_j) on A's
 * pattern (x = the forward solution).  With HZ_SYMMETRIC the caller
 * asserts A = A^T and the solve runs on conj(grad_x) with A itself;
 * otherwise A^H is formed in the workspace (deterministically: rows sorted
 * by column).  Synchronises the stream; returns the adjoint solve's status.
 */
int zbicgstab_adjoint(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                      const hz_c128 *vals, const hz_c128 *x, const hz_c128 *grad_x, hz_c128 *grad_b,
                      hz_c128 *grad_vals, double rtol, int maxiter, int flags, void *ws, size_t ws_bytes,
                      hz_solve_info *info);

/* Device workspace (bytes) that zbicgstab_adjoint_batched needs. */
size_t zbicgstab_adjoint_batched_workspace_bytes(int nsys, int n, int nnz, int flags);

/*
 * Backward of a shared-pattern batch x_j = A_j^{-1} b_j (zbicgstab_solve_batched,
 * same layout: vals [nnz][nsys], vectors [n][nsys]): for every system solve
 * A_j^H lambda_j = grad_x_j by the batched BiCGStab (rtol, maxiter,
 * HZ_PRECOND_JACOBI; zero initial guess), write grad_b = lambda and, if
 * grad_vals is not NULL, grad_vals[p*nsys + j] = -lambda_j[i] conj(x_j[c])
 * for entry p = (i, c).  With HZ_SYMMETRIC every A_j = A_j^T is asserted
 * and the solves run on conjugated right-hand sides; otherwise the
 * transposed pattern and each system's conjugate-transposed values are
 * formed in the workspace.  infos is a HOST array of nsys results of the
 * adjoint solves; returns the largest status.  Synchronises the stream.
 */
int zbicgstab_adjoint_batched(hz_handle *handle, hz_stream stream, int nsys, int n, int nnz, const int *row_ptr,
                              const int *col_idx, const hz_c128 *vals, const hz_c128 *x, const hz_c128 *grad_x,
                              hz_c128 *grad_b, hz_c128 *grad_vals, double rtol, int maxiter, int flags, void *ws,
                              size_t ws_bytes, hz_solve_info *infos);

/* Device workspace (bytes) for csr_level_order and csr_zpermute. */
size_t csr_reorder_workspace_bytes(int n, int nnz);

/*
 * Level-set (breadth-first) ordering of the pattern, a locality analysis of
 * this library (the paper stores matrices in the order they come, Section
 * 3.2).  A first search from node 0 picks the smallest index on its deepest
 * level as start; a second search from there gives each node its level
 * (distance in the graph of row i -> col_idx entries); perm[k] is the
 * caller's index of the k-th node in (level, caller's index) order, nodes
 * the search does not reach last in index order; inv[perm[k]] = k.  level
 * (nullable, n ints) receives the levels of the second search, -1 where
 * unreached.  All outputs are device arrays of n ints owned by the caller;
 * the result is a pure function of row_ptr/col_idx.  ws as returned by
 * csr_reorder_workspace_bytes, 256-byte aligned.  Synchronises the stream.
 */
int csr_level_order(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                    int *perm, int *inv, int *level, void *ws, size_t ws_bytes);

/*
 * B = P A P^T for the permutation perm (new -> old) with inverse inv: row k
 * of B is row perm[k] of A with every column c renumbered inv[c], columns
 * sorted within each row, values carried along.  Outputs row_ptr_out
 * (n+1), col_idx_out (nnz), vals_out (nnz) are caller-owned device arrays
 * that must not overlap the inputs.  Returns HZ_ERR_INVALID unless perm is
 * a permutation of 0..n-1 and inv its inverse (checked on the device).
 * ws as for csr_level_order.  Synchronises the stream.
 */
int csr_zpermute(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                 const hz_c128 *vals, const int *perm, const int *inv, int *row_ptr_out, int *col_idx_out,
                 hz_c128 *vals_out, void *ws, size_t ws_bytes);

/*
 * Memory-bandwidth calibration (measurement only; the paper repeats every
 * operation and averages its time, Section 3.3, and these give the ceiling
 * that the bandwidth-bound kernels above are compared against on the same
 * part).  hz_stream_read reads `bytes` bytes of buf (device, 16-byte aligned,
 * bytes a multiple of 16) as doubles, each thread keeping eight independent
 * non-temporal 16-byte loads in flight (32 KiB chunks, a few per block), and
 * writes their sum, in a fixed order, to *out (device double).  hz_stream_copy copies `bytes` bytes from src to dst
 * (device, 16-byte aligned, not overlapping) the same way.  Both enqueue on
 * the stream and return HZ_ERR_INVALID for bad pointers or sizes.  The read
 * uses the handle's partial-sum buffer: calls on one handle must not
 * overlap.
 */
int hz_stream_read(hz_handle *handle, hz_stream stream, const void *buf, size_t bytes, double *out);
int hz_stream_copy(hz_handle *handle, hz_stream stream, const void *src, void *dst, size_t bytes);

/*
 * Product in the caller's numbering through a renumbered copy (Section 3.2
 * CSR storage, Section 6 product; the renumbering is not the paper's, see
 * csr_level_order).  A randomly numbered matrix makes nearly every gathered
 * 16-byte x element fetch its own cache line; a plan keeps the level-set
 * renumbered copy P A P^T so that repeated products stream it instead.
 * csr_zspmv_plan builds the plan in caller-owned device memory `plan` of
 * csr_zspmv_plan_bytes(n, nnz) bytes (256-byte aligned; it holds perm and
 * its inverse (4 n each), P A P^T (20 nnz + 4 (n + 1)), room for P x (16 n)
 * and the ordering scratch) and synchronises the stream.  The plan copies
 * the values: after the caller changes vals it must be rebuilt.
 * csr_zspmv_planned computes y = A x (caller's numbering) as x_p = P x
 * (gathered once), then the block-tile product of P A P^T writing row k to
 * y[perm[k]] (about 72 n bytes more than csr_zspmv moves, for gathers that
 * stay in cache).  n and nnz must be those the plan was built with; x and y
 * must not overlap each other or the plan.  Concurrent products on one plan
 * race on its x_p.  Returns HZ_ERR_WORKSPACE for a missing, misaligned or
 * small plan, HZ_ERR_INVALID for bad pointers or overlaps.
 */
size_t csr_zspmv_plan_bytes(int n, int nnz);
int csr_zspmv_plan(hz_handle *handle, hz_stream stream, int n, int nnz, const int *row_ptr, const int *col_idx,
                   const hz_c128 *vals, void *plan, size_t plan_bytes);
int csr_zspmv_planned(hz_handle *handle, hz_stream stream, int n, int nnz, const void *plan, size_t plan_bytes,
                      const hz_c128 *x, hz_c128 *y);

#ifdef __cplusplus
}
#endif
#endif /* HELMZ_H */
