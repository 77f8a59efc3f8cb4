"""Python face of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  It wraps the plain C oracle
(``krylov.c``, ``refine.c``; sequential complex arithmetic compiled without
FMA contraction) and adds dense numpy references (LAPACK LU) used to pin the
oracle itself.  Nothing here imports or loads the GPU library.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE, INVALID = 0, 1, 2, 3, -1
STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", BREAKDOWN: "BREAKDOWN", NONFINITE: "NONFINITE", INVALID: "INVALID"}


class _Z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class _C(C.Structure):
    _fields_ = [("re", C.c_float), ("im", C.c_float)]


class _Info(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("iterations", C.c_int),
        ("outer_steps", C.c_int),
        ("pad", C.c_int),
        ("relres_recursive", C.c_double),
        ("relres_true", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {
            "status": self.status,
            "iterations": self.iterations,
            "outer_steps": self.outer_steps,
            "relres_recursive": self.relres_recursive,
            "relres_true": self.relres_true,
        }


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _build.stale():
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        for pfx, S, R in (("z", _Z, C.c_double), ("c", _C, C.c_float)):
            getattr(L, f"or_{pfx}spmv").argtypes = [C.c_int, P, P, P, P, P]
            getattr(L, f"or_{pfx}dotc").argtypes = [C.c_int, P, P]
            getattr(L, f"or_{pfx}dotc").restype = S
            getattr(L, f"or_{pfx}nrm2").argtypes = [C.c_int, P]
            getattr(L, f"or_{pfx}nrm2").restype = R
            getattr(L, f"or_{pfx}axpy").argtypes = [C.c_int, S, P, P]
            getattr(L, f"or_{pfx}scal").argtypes = [C.c_int, S, P]
            getattr(L, f"or_{pfx}xmy").argtypes = [C.c_int, P, P]
            getattr(L, f"or_{pfx}bicgstab_work_elems").argtypes = [C.c_int]
            getattr(L, f"or_{pfx}bicgstab_work_elems").restype = C.c_size_t
            getattr(L, f"or_{pfx}bicgstab").argtypes = [
                C.c_int, P, P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int, P, C.POINTER(_Info)
            ]
            getattr(L, f"or_{pfx}bicgstab").restype = C.c_int
        L.or_zbicgstab_mixed.argtypes = [
            C.c_int, P, P, P, P, P, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(_Info)
        ]
        L.or_zbicgstab_mixed.restype = C.c_int
        L.or_zcsr_conj_transpose.argtypes = [C.c_int, P, P, P, P, P, P]
        L.or_zgrad_vals.argtypes = [C.c_int, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(A, cdtype=np.complex128):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    v = np.ascontiguousarray(A.vals, dtype=cdtype)
    return rp, ci, v


# ---------------------------------------------------------------- kernels


def zspmv(A, x: np.ndarray) -> np.ndarray:
    """y = A x (CSR, Section 3.2), complex128."""
    rp, ci, v = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty(A.n, dtype=np.complex128)
    lib().or_zspmv(A.n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def cspmv(A, x: np.ndarray) -> np.ndarray:
    """y = A x with A's values and x rounded to complex64, complex64 arithmetic."""
    rp, ci, v = _csr(A, np.complex64)
    x = np.ascontiguousarray(x, dtype=np.complex64)
    y = np.empty(A.n, dtype=np.complex64)
    lib().or_cspmv(A.n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def zdotc(x: np.ndarray, y: np.ndarray) -> complex:
    """sum conj(x_i) y_i (Section 5)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    r = lib().or_zdotc(x.shape[0], _p(x), _p(y))
    return complex(r.re, r.im)


def dznrm2(x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return float(lib().or_znrm2(x.shape[0], _p(x)))


def zaxpy(alpha: complex, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Returns alpha x + y (y is not modified)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.array(y, dtype=np.complex128, copy=True)
    lib().or_zaxpy(x.shape[0], _Z(alpha.real, alpha.imag), _p(x), _p(out))
    return out


def zscal(alpha: complex, x: np.ndarray) -> np.ndarray:
    out = np.array(x, dtype=np.complex128, copy=True)
    lib().or_zscal(out.shape[0], _Z(alpha.real, alpha.imag), _p(out))
    return out


def zxmy(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.array(y, dtype=np.complex128, copy=True)
    lib().or_zxmy(x.shape[0], _p(x), _p(out))
    return out


# ---------------------------------------------------------------- solvers


def zbicgstab(A, b, tol=1e-8, maxiter=20000, jacobi=False, x0=None):
    """Preconditioned BiCGStab in complex128 (Section 7).  Returns (x, info)."""
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros(A.n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    work = np.empty(lib().or_zbicgstab_work_elems(A.n), dtype=np.complex128)
    info = _Info()
    lib().or_zbicgstab(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), tol, maxiter, int(jacobi), int(x0 is None), _p(work), C.byref(info))
    return x, info.as_dict()


def cbicgstab(A, b, tol=1e-4, maxiter=20000, jacobi=False):
    """The same algorithm instantiated in complex64."""
    rp, ci, v = _csr(A, np.complex64)
    b = np.ascontiguousarray(b, dtype=np.complex64)
    x = np.zeros(A.n, dtype=np.complex64)
    work = np.empty(lib().or_cbicgstab_work_elems(A.n), dtype=np.complex64)
    info = _Info()
    lib().or_cbicgstab(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), tol, maxiter, int(jacobi), 1, _p(work), C.byref(info))
    return x, info.as_dict()


def zbicgstab_mixed(A, b, tol=1e-10, inner_tol=1e-4, maxiter=20000, max_outer=50, jacobi=False):
    """Complex64-inner / complex128-refinement solve.  Returns (x, info)."""
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros(A.n, dtype=np.complex128)
    info = _Info()
    lib().or_zbicgstab_mixed(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), tol, inner_tol, maxiter, max_outer, int(jacobi), C.byref(info))
    return x, info.as_dict()


def zbicgstab_batched(systems, tol=1e-8, maxiter=20000, jacobi=False):
    """A loop of independent single solves; ``systems`` is a list of (A, b)."""
    return [zbicgstab(A, b, tol=tol, maxiter=maxiter, jacobi=jacobi) for A, b in systems]


def zcsr_conj_transpose(A):
    from workloads.csr import CSR  # input container only

    rp, ci, v = _csr(A)
    trp = np.empty(A.n + 1, dtype=np.int32)
    tci = np.empty(A.nnz, dtype=np.int32)
    tv = np.empty(A.nnz, dtype=np.complex128)
    lib().or_zcsr_conj_transpose(A.n, _p(rp), _p(ci), _p(v), _p(trp), _p(tci), _p(tv))
    return CSR(trp, tci, tv)


def zgrad_vals(A, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """grad of entry (i, j) = -lambda_i conj(x_j), on A's pattern."""
    rp, ci, _ = _csr(A)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    g = np.empty(A.nnz, dtype=np.complex128)
    lib().or_zgrad_vals(A.n, _p(rp), _p(ci), _p(lam), _p(x), _p(g))
    return g


def zadjoint(A, x, grad_x, tol=1e-10, maxiter=20000, jacobi=False):
    """Backward of x = A^{-1} b: solve A^H lambda = grad_x, then entry gradients.

    Returns (grad_b = lambda, grad_vals, info).  Uses an explicit conjugate
    transpose, so it does not rely on A = A^T.
    """
    AH = zcsr_conj_transpose(A)
    lam, info = zbicgstab(AH, grad_x, tol=tol, maxiter=maxiter, jacobi=jacobi)
    return lam, zgrad_vals(A, lam, x), info


# ---------------------------------------------------------------- dense references (numpy / LAPACK)


def to_dense(A) -> np.ndarray:
    D = np.zeros((A.n, A.n), dtype=np.complex128)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    D[rows, A.col_idx] = A.vals
    return D


def dense_solve(A, b) -> np.ndarray:
    """LAPACK LU solve (zgesv through numpy)."""
    return np.linalg.solve(to_dense(A), np.asarray(b, dtype=np.complex128))


def threads_used() -> int:
    """Threads of the sequential oracle (the functions above)."""
    return 1


# ---------------------------------------------------------------- threaded build (timing only)

_omp = None


def omp_lib():
    """The OpenMP build of the complex128 oracle (liboracle_omp.so), for timing on all host cores."""
    global _omp
    if _omp is None:
        lib()  # builds both libraries when stale
        L = C.CDLL(_build.LIB_OMP)
        P = C.c_void_p
        L.or_zspmv.argtypes = [C.c_int, P, P, P, P, P]
        L.or_zbicgstab_work_elems.argtypes = [C.c_int]
        L.or_zbicgstab_work_elems.restype = C.c_size_t
        L.or_zbicgstab.argtypes = [C.c_int, P, P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int, P, C.POINTER(_Info)]
        L.or_zbicgstab.restype = C.c_int
        _omp = L
    return _omp


def omp_threads() -> int:
    """Threads the OpenMP build runs with (OMP_NUM_THREADS, else the affinity cores)."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else affinity_cores()


def zspmv_omp(A, x: np.ndarray) -> np.ndarray:
    """y = A x by the threaded build (rows split across threads; every row sums as in zspmv)."""
    rp, ci, v = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty(A.n, dtype=np.complex128)
    omp_lib().or_zspmv(A.n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def zbicgstab_omp(A, b, x0=None, tol=1e-8, maxiter=20000, jacobi=False):
    """zbicgstab by the threaded build: the same algorithm, dot products summed per thread."""
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros(A.n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    L = omp_lib()
    work = np.empty(L.or_zbicgstab_work_elems(A.n), dtype=np.complex128)
    info = _Info()
    L.or_zbicgstab(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), float(tol), int(maxiter), int(bool(jacobi)),
                   int(x0 is None), _p(work), C.byref(info))
    return x, info.as_dict()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def affinity_cores() -> int:
    return len(os.sched_getaffinity(0))
