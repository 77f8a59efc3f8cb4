"""BiCGstab(l) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  The paper runs a preconditioned
BiCGSTAB(l) with l = 8 beside P-BiCGSTAB (Section 7, iterative Krylov
methods, and its speed-up tables for Audi3D, Twingo3D and Cylinder3D) without
printing the algorithm; this is the method of Sleijpen and Fokkema (1993),
written from its published steps in complex128:

* a cycle makes l Bi-CG steps, keeping the residuals r_0..r_l and the search
  directions u_0..u_l of one step apart in powers of the operator
  (r_{i+1} = A r_i, u_{i+1} = A u_i), with the scalars rho, alpha, beta of
  Bi-CG and the fixed shadow residual r~ = r_0 of the first cycle;
* then the minimal-residual part takes the coefficients gamma_1..gamma_l that
  minimise || r_0 - sum_j gamma_j r_j ||_2 (this module calls numpy's
  least-squares solver: the minimiser has this plain definition, whichever
  orthogonalisation computes it), and updates
  x += sum_j gamma_j r_{j-1},  r_0 -= sum_j gamma_j r_j,  u_0 -= sum_j gamma_j u_j,
  omega = gamma_l (the next cycle starts from rho_0 = -omega rho_0).

Right preconditioning with M = diag(A) is applied as for BiCGStab: the
iteration runs on A D^{-1} y = b and returns x = D^{-1} y.  Inner products
are <a, b> = sum conj(a_i) b_i.  Convergence is tested on the recursive
residual at the end of every cycle; `info["iterations"]` counts cycles (each
cycle is l Bi-CG steps and 2 l products).  A breakdown is an exact zero
rho or <r~, u_{j+1}>, or a rank-deficient minimal-residual system.
"""

from __future__ import annotations

import numpy as np

from .oracle import zspmv

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def _dot(a, b):
    return complex(np.vdot(a, b))  # sum conj(a_i) b_i


def bicgstab_l(A, b, ell=8, tol=1e-8, maxcycles=2000, jacobi=False, x0=None, trace=None):
    """Solve A x = b by BiCGstab(ell).  Returns (x, info).

    ``trace(cycle, rhat, uhat, r_new, y_new)``, if given, is called after each
    cycle's minimal-residual part with the Bi-CG bases of the cycle (lists of
    ell + 1 vectors, before the update) and the new residual and iterate (of
    the preconditioned system).
    """
    n = A.n
    b = np.asarray(b, dtype=np.complex128)
    if jacobi:
        diag = np.zeros(n, dtype=np.complex128)
        rows = A.row_of_entry()
        on = A.col_idx == rows
        diag[rows[on]] = A.vals[on]
        dinv = 1.0 / diag
    else:
        dinv = None

    def op(v):
        return zspmv(A, dinv * v if jacobi else v)

    bn = float(np.linalg.norm(b))
    info = {"status": OK, "iterations": 0, "relres_recursive": 0.0, "relres_true": 0.0}
    if bn == 0.0:
        return np.zeros(n, dtype=np.complex128), info
    if x0 is None:
        y = np.zeros(n, dtype=np.complex128)
        r = b.copy()
    else:
        x0 = np.asarray(x0, dtype=np.complex128)
        y = x0 / dinv if jacobi else x0.copy()
        r = b - zspmv(A, x0)
    rt = r.copy()  # shadow residual
    u = np.zeros(n, dtype=np.complex128)
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    relres = float(np.linalg.norm(r)) / bn
    status = NOT_CONVERGED
    cycles = 0
    if relres <= tol:
        status = OK
    while status == NOT_CONVERGED and cycles < maxcycles:
        rhat = [r] + [None] * ell
        uhat = [u] + [None] * ell
        rho0 = -omega * rho0
        bad = None
        for j in range(ell):  # Bi-CG part
            rho1 = _dot(rt, rhat[j])
            if rho0 == 0 or rho1 == 0:
                bad = BREAKDOWN
                break
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                uhat[i] = rhat[i] - beta * uhat[i]
            uhat[j + 1] = op(uhat[j])
            gamma = _dot(rt, uhat[j + 1])
            if gamma == 0:
                bad = BREAKDOWN
                break
            alpha = rho0 / gamma
            for i in range(j + 1):
                rhat[i] = rhat[i] - alpha * uhat[i + 1]
            rhat[j + 1] = op(rhat[j])
            y = y + alpha * uhat[0]
        if bad is not None:
            status = bad
            r = rhat[0]
            break
        R = np.column_stack(rhat[1:])
        g, _, rank, _ = np.linalg.lstsq(R, rhat[0], rcond=None)
        if rank < ell or not np.all(np.isfinite(g)):
            status = BREAKDOWN if np.all(np.isfinite(g)) else NONFINITE
            r = rhat[0]
            break
        omega = complex(g[-1])
        y = y + np.column_stack(rhat[:ell]) @ g
        r = rhat[0] - R @ g
        u = uhat[0] - np.column_stack(uhat[1:]) @ g
        cycles += 1
        if trace is not None:
            trace(cycles, rhat, uhat, r, y)
        relres = float(np.linalg.norm(r)) / bn
        if not np.isfinite(relres):
            status = NONFINITE
        elif relres <= tol:
            status = OK
    x = dinv * y if jacobi else y
    info["status"] = status
    info["iterations"] = cycles
    info["relres_recursive"] = relres
    info["relres_true"] = float(np.linalg.norm(b - zspmv(A, x))) / bn
    return x, info
