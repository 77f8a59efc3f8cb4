"""Pins of the oracle's TFQMR against what the method and linear algebra fix.

- TFQMR is built on CGS: after every odd half step m, w_{m+1} = w_{2k} is the
  k-th residual of a textbook CGS written in this test;
- the quasi-minimal-residual bound ||b - A x_{m+1}|| <= sqrt(m + 2) tau_{m+1}
  holds after every half step, and tau never grows;
- the iterates are the QMR smoothing of the w sequence: 1/tau_m^2 =
  sum_j 1/||w_j||^2, and r_{m+1} = (1 - c^2) r_m + c^2 w_{m+1} for the true
  residuals, c^2 = tau_{m+1}^2 / ||w_{m+1}||^2;
- A = s I is solved in one iteration (x = b / s);
- converged solutions agree with dense LU; Jacobi equals the plain method on
  the explicitly column-scaled matrix; b = 0 and an exact x0.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.tfqmr import tfqmr
from workloads.csr import CSR, csr_from_coo


def dense_csr(D):
    n = D.shape[0]
    r, c = np.nonzero(D != 0)
    return csr_from_coo(n, r, c, D[r, c].astype(np.complex128))


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def cgs_residuals(D, b, k):
    """Textbook CGS (Sonneveld), shadow r~ = b: residuals r_0 .. r_k."""
    r = b.copy()
    rt = r.copy()
    p, u = r.copy(), r.copy()
    rho = np.vdot(rt, r)
    out = [r.copy()]
    for _ in range(k):
        v = D @ p
        alpha = rho / np.vdot(rt, v)
        q = u - alpha * v
        r = r - alpha * (D @ (u + q))
        rho_new = np.vdot(rt, r)
        beta = rho_new / rho
        u = r + beta * q
        p = u + beta * (q + beta * p)
        rho = rho_new
        out.append(r.copy())
    return out


@pytest.mark.parametrize("jacobi", [False, True])
def test_even_w_are_cgs_residuals_and_the_bound_holds(jacobi):
    rng = np.random.default_rng(3)
    n = 50
    D = cn(rng, n, n) / np.sqrt(n) + 5 * np.eye(n)
    D[np.arange(n), np.arange(n)] *= 1 + 0.3j
    b = cn(rng, n)
    dinv = 1.0 / np.diag(D) if jacobi else np.ones(n)
    Dh = D * dinv[None, :]
    rc = cgs_residuals(Dh, b, 6)
    taus, errs, bounds, harm, smooth = [], [], [], [], []
    st = {"x": np.zeros(n, complex), "inv": 1 / np.linalg.norm(b) ** 2}

    def trace(m, w, x, tau):
        if m % 2 == 1 and (m + 1) // 2 < len(rc):
            k = (m + 1) // 2
            errs.append(np.linalg.norm(w - rc[k]) / np.linalg.norm(rc[k]))
        bounds.append(np.linalg.norm(b - D @ x) / (np.sqrt(m + 2) * tau))
        taus.append(tau)
        # QMR smoothing of the w sequence (Zhou and Walker): 1/tau_m^2 = sum_j 1/||w_j||^2
        # (w_0 = r_0), and the true residuals obey r_{m+1} = (1 - c^2) r_m + c^2 w_{m+1}
        # with c^2 = tau_{m+1}^2 / ||w_{m+1}||^2
        nw = np.linalg.norm(w)
        st["inv"] += 1 / nw**2
        harm.append(abs(1 / tau**2 - st["inv"]) * tau**2)
        c2 = tau**2 / nw**2
        r_prev, r_new = b - D @ st["x"], b - D @ x
        smooth.append(np.linalg.norm(r_new - ((1 - c2) * r_prev + c2 * w)) / np.linalg.norm(b))
        st["x"] = x

    x, info = tfqmr(dense_csr(D), b, tol=1e-12, jacobi=jacobi, trace=trace)
    assert info["status"] == O.OK
    assert len(errs) >= 4 and max(errs) <= 1e-10, errs
    assert max(bounds) <= 1 + 1e-8
    assert max(harm) <= 1e-12 and max(smooth) <= 1e-12, (max(harm), max(smooth))
    assert all(t2 <= t1 * (1 + 1e-15) for t1, t2 in zip(taus, taus[1:]))
    xd = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_scaled_identity_in_one_iteration():
    n = 20
    s = 2.0 - 0.5j
    A = dense_csr(s * np.eye(n))
    b = cn(np.random.default_rng(1), n)
    x, info = tfqmr(A, b, tol=1e-14)
    assert info["status"] == O.OK and info["iterations"] == 1
    assert np.allclose(x, b / s, rtol=1e-15, atol=1e-15)


def test_helmholtz_cube_matches_dense_lu():
    A, b, _ = W.config_cube(7, seed=1)
    x, info = tfqmr(A, b, tol=1e-11)
    assert info["status"] == O.OK
    assert info["relres_true"] <= 1e-11
    xd = np.linalg.solve(O.to_dense(A), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_jacobi_equals_plain_method_on_scaled_matrix():
    A, b, _ = W.config_cylinder(h=0.25)
    diag = np.zeros(A.n, complex)
    rows = A.row_of_entry()
    on = A.col_idx == rows
    diag[rows[on]] = A.vals[on]
    S = CSR(A.row_ptr, A.col_idx, A.vals / diag[A.col_idx])  # A D^{-1}
    xj, ij = tfqmr(A, b, tol=1e-30, maxiter=12, jacobi=True)
    ys, iy = tfqmr(S, b, tol=1e-30, maxiter=12)
    assert ij["iterations"] == iy["iterations"] == 12
    assert np.linalg.norm(xj - ys / diag) <= 1e-11 * np.linalg.norm(xj)


def test_special_cases():
    A, b, _ = W.config_cube(5, seed=3)
    x, info = tfqmr(A, np.zeros(A.n, complex))
    assert info["status"] == O.OK and info["iterations"] == 0 and not np.any(x)
    xd = np.linalg.solve(O.to_dense(A), b)
    x, info = tfqmr(A, b, tol=1e-8, x0=xd)
    assert info["status"] == O.OK and info["iterations"] == 0
    x, info = tfqmr(A, b, tol=1e-12, x0=0.5 * xd)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-12
