"""Mixed-precision BiCGStab with reliable updates -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  An extension of the paper's
P-BiCGSTAB (Section 7), not in the paper: the Krylov iteration runs in a
lower precision (complex64) on the scaled problem A D^{-1} y = b / ||b||, and
the accuracy comes from reliable updates in the sense of Sleijpen and van der
Vorst ("Reliable updated residuals in hybrid Bi-CG methods", Computing 56,
1996): whenever the recursive residual of the low-precision iteration has
fallen by a factor `delta` since the last update (or the iteration budget is
spent),

* the iterate is flushed to complex128: x <- x + ||b|| D^{-1} y, y <- 0;
* the true residual b - A x is formed in complex128 and decides convergence
  (||b - A x|| / ||b|| <= tol);
* the low-precision recursive residual is replaced by (b - A x) / ||b||,
  while the search directions p, v, the shadow residual and the scalars
  carry on (no restart of the Krylov space).

The iteration itself is the textbook right-preconditioned BiCGStab (the
oracle's `zbicgstab` in oracle/krylov.c, written independently): with
rho = <r~, r>, beta = (rho / rho_prev)(alpha / omega),
p = r + beta (p - omega v), v = A D^{-1} p, alpha = rho / <r~, v>,
s = r - alpha v, t = A D^{-1} s, omega = <t, s> / <t, t>,
y <- y + alpha p + omega s, r = s - omega t (y solves the scaled problem, so
x = ||b|| D^{-1} y).  Vectors and the
product are in the inner precision (A's values and D^{-1} rounded to it;
the products through the oracle's own complex64 / complex128 SpMV); the
scalars and the sums of the inner products are complex128 (one of the two
readings of the extension that the checks accept, the other accumulating in
complex64).  Starting guess zero.  With `inner=np.complex128` the same steps
run in double precision and the iteration counts to a given tolerance are
those of the textbook solver within a step or two (the reliable update then
only replaces r by the equal-in-exact-arithmetic true residual).

Returns (x, info) with info = {status, iterations, outer_steps (the
number of reliable updates), relres_true}; status 0 = converged,
1 = not converged within maxiter, 2 = breakdown (an exact zero rho or
<r~, v>, or <t, t> = 0 with s != 0).  An exactly zero s (the half step
solved the inner problem) takes y += alpha p and a reliable update.
"""

from __future__ import annotations

import numpy as np

from .oracle import cspmv, zspmv


def _diag(A) -> np.ndarray:
    d = np.zeros(A.n, dtype=np.complex128)
    for i in range(A.n):
        for p in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            if int(A.col_idx[p]) == i:
                d[i] = A.vals[p]
    return d


def _dot(a: np.ndarray, b: np.ndarray) -> complex:
    """sum conj(a_i) b_i accumulated in complex128 (sequential order)."""
    return complex(np.sum(np.conj(a.astype(np.complex128)) * b.astype(np.complex128)))


def zbicgstab_reliable(A, b, tol=1e-10, delta=0.1, maxiter=20000, jacobi=False, inner=np.complex64):
    b = np.asarray(b, dtype=np.complex128)
    n = A.n
    x = np.zeros(n, dtype=np.complex128)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return x, {"status": 0, "iterations": 0, "outer_steps": 0, "relres_true": 0.0}
    prod = zspmv if inner == np.complex128 else cspmv
    if jacobi:
        d = _diag(A)
        if np.any(d == 0):
            raise ValueError("Jacobi needs a nonzero diagonal")
        dinv = (1.0 / d).astype(inner)
    else:
        dinv = np.ones(n, dtype=inner)

    def op(w):  # A D^{-1} w in the inner precision
        return prod(A, (dinv * w).astype(inner)).astype(inner)

    r = (b / bn).astype(inner)
    rt = r.copy()
    p = np.zeros(n, dtype=inner)
    v = np.zeros(n, dtype=inner)
    y = np.zeros(n, dtype=inner)
    rho_prev = alpha = omega = 1.0 + 0.0j
    r_ref = float(np.linalg.norm(r.astype(np.complex128)))
    updates = 0
    rel = 1.0
    status = 1
    it = 0

    def flush():
        nonlocal x, y, rel, updates
        x = x + bn * (dinv.astype(np.complex128) * y.astype(np.complex128))
        y = np.zeros(n, dtype=inner)
        r64 = b - zspmv(A, x)
        rel = float(np.linalg.norm(r64)) / bn
        updates += 1
        return r64

    c = lambda z: inner(z)  # noqa: E731  (a complex128 scalar rounded to the inner precision)
    while it < maxiter:
        it += 1
        rho = _dot(rt, r)
        if rho == 0:
            status = 2
            break
        beta = (rho / rho_prev) * (alpha / omega)
        p = (r + c(beta) * (p - c(omega) * v)).astype(inner)
        v = op(p)
        sigma = _dot(rt, v)
        if sigma == 0:
            status = 2
            break
        alpha = rho / sigma
        s = (r - c(alpha) * v).astype(inner)
        if not np.any(s):  # the half step solved the inner problem exactly: x takes alpha p, then an update
            y = (y + c(alpha) * p).astype(inner)
            r64 = flush()
            if rel <= tol:
                status = 0
                break
            r = (r64 / bn).astype(inner)
            r_ref = float(np.linalg.norm(r.astype(np.complex128)))
            rho_prev = rho
            continue
        t = op(s)
        tt = _dot(t, t).real
        if tt == 0:
            status = 2
            break
        omega = _dot(t, s) / tt
        y = (y + c(alpha) * p + c(omega) * s).astype(inner)
        r = (s - c(omega) * t).astype(inner)
        rho_prev = rho
        rn = float(np.linalg.norm(r.astype(np.complex128)))
        if rn <= delta * r_ref or it == maxiter:
            r64 = flush()
            if rel <= tol:
                status = 0
                break
            r = (r64 / bn).astype(inner)
            r_ref = float(np.linalg.norm(r.astype(np.complex128)))
    if status != 0 and np.any(y != 0):
        flush()
        if rel <= tol:
            status = 0
    return x, {"status": status, "iterations": it, "outer_steps": updates, "relres_true": rel}
