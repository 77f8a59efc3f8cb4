"""Transpose-free QMR -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  The paper runs a preconditioned
transpose-free QMR (P-TFQMR; "P-QMR" in its Cylinder3D table) beside
P-BiCGSTAB, citing Saad's book for its solvers (Section 7, iterative Krylov
methods, and its speed-up tables), without printing the algorithm.  This is
Freund's TFQMR in the form of Saad's "Iterative methods for sparse linear
systems", written from its steps in complex128, with half steps m = 0, 1, ...:

* even m: alpha = rho_m / <r~, v_m>, u_{m+1} = u_m - alpha v_m;
* every m: w_{m+1} = w_m - alpha A u_m;
  d_{m+1} = u_m + (theta_m^2 / alpha) eta_m d_m;
  theta_{m+1} = ||w_{m+1}|| / tau_m, c = (1 + theta_{m+1}^2)^(-1/2),
  tau_{m+1} = tau_m theta_{m+1} c, eta_{m+1} = c^2 alpha;
  x_{m+1} = x_m + eta_{m+1} d_{m+1};
* odd m: rho_{m+1} = <r~, w_{m+1}>, beta = rho_{m+1} / rho_{m-1},
  u_{m+1} = w_{m+1} + beta u_m,
  v_{m+1} = A u_{m+1} + beta (A u_m + beta v_{m-1});

from w_0 = u_0 = r_0 = b - A x_0, v_0 = A u_0, d_0 = 0, tau_0 = ||r_0||,
theta_0 = eta_0 = 0 and r~ = r_0.  Inner products are <a, b> = sum conj(a_i) b_i;
theta, c and tau are real, alpha, eta, rho, beta complex.  Right Jacobi
preconditioning as for BiCGStab (the iteration runs on A D^{-1}).

Stopping (reading of the paper's residual threshold): the quasi-residual
bound ||b - A x_{m+1}|| <= sqrt(m + 2) tau_{m+1} <= tol ||b||, tested after
every half step; `info["iterations"]` counts full iterations (two half
steps, two products; an exit after the first half step of an iteration
counts it).  A breakdown is an exact zero <r~, v_m> or rho_{m-1}.
"""

from __future__ import annotations

import math

import numpy as np

from .oracle import zspmv

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def _dot(a, b):
    return complex(np.vdot(a, b))  # sum conj(a_i) b_i


def tfqmr(A, b, tol=1e-8, maxiter=20000, jacobi=False, x0=None, trace=None):
    """Solve A x = b by TFQMR.  Returns (x, info).

    ``trace(m, w, x_of_m_plus_1, tau)`` is called after every half step m
    with w_{m+1}, the iterate x_{m+1} of the original system and tau_{m+1}.
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

    def orig(y):
        return dinv * y if jacobi else y

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
    rt = r.copy()
    w, u = r.copy(), r.copy()
    Au = op(u)
    v = Au.copy()
    d = np.zeros(n, dtype=np.complex128)
    tau = float(np.linalg.norm(r))
    theta, eta = 0.0, 0j
    rho = _dot(rt, r)
    alpha = 0j
    status = NOT_CONVERGED
    bound = tau / bn
    half = 0
    if bound <= tol:
        status = OK
    v_prev = None  # v_{m-1} at odd m
    while status == NOT_CONVERGED and half < 2 * maxiter:
        m = half
        if m % 2 == 0:
            sigma = _dot(rt, v)
            if sigma == 0:
                status = BREAKDOWN
                break
            alpha = rho / sigma
            u_next = u - alpha * v
            v_prev = v
        w = w - alpha * Au
        d = u + (theta * theta / alpha) * eta * d
        theta = float(np.linalg.norm(w)) / tau
        c = 1.0 / math.sqrt(1.0 + theta * theta)
        tau = tau * theta * c
        eta = c * c * alpha
        y = y + eta * d
        if trace is not None:
            trace(m, w, orig(y), tau)
        half += 1
        bound = math.sqrt(m + 2) * tau / bn
        if not math.isfinite(bound):
            status = NONFINITE
            break
        if bound <= tol:
            status = OK
            break
        if m % 2 == 0:
            u = u_next
            Au = op(u)  # A u_{m+1}: the product of the odd half step
        else:
            rho_new = _dot(rt, w)
            if rho == 0:
                status = BREAKDOWN
                break
            beta = rho_new / rho
            rho = rho_new
            u_odd, Au_odd = u, Au
            u = w + beta * u_odd
            Au = op(u)
            v = Au + beta * (Au_odd + beta * v_prev)
    x = orig(y)
    info["status"] = status
    info["iterations"] = (half + 1) // 2
    info["relres_recursive"] = bound
    info["relres_true"] = float(np.linalg.norm(b - zspmv(A, x))) / bn
    return x, info
