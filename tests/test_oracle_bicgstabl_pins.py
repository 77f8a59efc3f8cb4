"""Pins of the oracle's BiCGstab(l) against what the method and linear algebra fix.

- l = 1 is BiCGStab: its iterates equal those of the oracle's (independent, C)
  BiCGStab after the same number of iterations;
- after every cycle's Bi-CG part the bases satisfy r_j = A r_{j-1} and
  u_j = A u_{j-1} (checked with a dense product), and the minimal-residual
  update leaves a residual orthogonal to r_1..r_l (to rounding scaled by the
  basis' condition number) that equals b - A y;
- the Bi-CG part of cycle k leaves r_0 = psi_{k-1}(A) phi_{kl}(A) r_0, with phi
  the residual polynomial of a textbook Bi-CG written in the test and psi the
  earlier cycles' minimal-residual polynomials;
- with l at least the number of distinct eigenvalues one cycle solves the
  system (Bi-CG terminates);
- converged solutions agree with dense LU; Jacobi equals the plain method on
  the explicitly column-scaled matrix; special cases b = 0 and an exact x0.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.bicgstabl import bicgstab_l
from workloads.csr import CSR, csr_from_coo


def dense_csr(D):
    n = D.shape[0]
    r, c = np.nonzero(D != 0)
    return csr_from_coo(n, r, c, D[r, c].astype(np.complex128))


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_system(n=60, seed=0, shift=6.0):
    rng = np.random.default_rng(seed)
    D = cn(rng, n, n) / np.sqrt(n) + shift * np.eye(n)
    return D, cn(rng, n)


@pytest.mark.parametrize("jacobi", [False, True])
def test_l1_reproduces_bicgstab_iterates(jacobi):
    A, b, _ = W.config_cube(6, seed=2)
    for k in (1, 3, 7):
        xs, inf_s = O.zbicgstab(A, b, tol=1e-30, maxiter=k, jacobi=jacobi)
        xl, inf_l = bicgstab_l(A, b, ell=1, tol=1e-30, maxcycles=k, jacobi=jacobi)
        assert inf_s["iterations"] == k and inf_l["iterations"] == k
        assert np.linalg.norm(xl - xs) <= 1e-10 * np.linalg.norm(xs), k


@pytest.mark.parametrize("ell", [2, 4, 8])
@pytest.mark.parametrize("jacobi", [False, True])
def test_cycle_relations_and_minimal_residual(ell, jacobi):
    D, b = random_system(seed=ell)
    D[np.arange(60), np.arange(60)] *= 1 + 0.5j  # a diagonal worth scaling
    A = dense_csr(D)
    dinv = 1.0 / np.diag(D) if jacobi else np.ones(60)
    Ah = D * dinv[None, :]  # the operator the iteration runs on
    seen = []

    def trace(cycle, rhat, uhat, r_new, y_new):
        # rounding scale: the largest basis vector of the cycle (the bases are
        # updated by differences of much larger terms); a wrong index or sign
        # breaks a relation by O(1) relative
        na = np.linalg.norm(Ah)
        rs = max(np.linalg.norm(v) for v in rhat)
        us = max(np.linalg.norm(v) for v in uhat)
        for j in range(1, ell + 1):
            assert np.linalg.norm(rhat[j] - Ah @ rhat[j - 1]) <= 1e-10 * na * rs
            assert np.linalg.norm(uhat[j] - Ah @ uhat[j - 1]) <= 1e-10 * na * us
        # least squares: r_new is orthogonal to r_1..r_l, to rounding that grows
        # with the conditioning of that (power-like) basis, on the scale of r_0
        R = np.column_stack(rhat[1:])
        sv = np.linalg.svd(R, compute_uv=False)
        ortho = np.abs(R.conj().T @ r_new) / (np.linalg.norm(R, axis=0) * np.linalg.norm(rhat[0]))
        assert ortho.max() <= 10 * np.finfo(float).eps * sv[0] / sv[-1], (ortho.max(), sv[0] / sv[-1])
        assert np.linalg.norm(r_new - (b - Ah @ y_new)) <= 1e-9 * np.linalg.norm(b)
        seen.append(cycle)

    x, info = bicgstab_l(A, b, ell=ell, tol=1e-12, jacobi=jacobi, trace=trace)
    assert info["status"] == O.OK and seen == list(range(1, info["iterations"] + 1))
    xd = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def bicg_residuals(D, b, m):
    """Textbook Bi-CG (shadow system with D^H, shadow start = b): residuals r_0..r_m."""
    r, rt = b.copy(), b.copy()
    p, pt = r.copy(), rt.copy()
    rho = np.vdot(rt, r)
    out = [r.copy()]
    for _ in range(m):
        q, qt = D @ p, D.conj().T @ pt
        alpha = rho / np.vdot(pt, q)
        r = r - alpha * q
        rt = rt - np.conj(alpha) * qt
        rho_new = np.vdot(rt, r)
        beta = rho_new / rho
        p = r + beta * p
        pt = rt + np.conj(beta) * pt
        rho = rho_new
        out.append(r.copy())
    return out


@pytest.mark.parametrize("ell", [2, 3])
def test_bicg_part_is_bicg_times_earlier_minimal_residual_polynomials(ell):
    """At the end of cycle k's Bi-CG part, r_0 = psi_{k-1}(A) phi_{k l}(A) r_0 (Sleijpen and
    Fokkema): phi the Bi-CG residual polynomial (from the textbook Bi-CG above), psi the
    product of the earlier cycles' minimal-residual polynomials 1 - sum_j gamma_j t^j, whose
    gamma are read back from each traced update (R gamma = r_0 - r_new)."""
    D, b = random_system(n=50, seed=20 + ell, shift=5.0)
    A = dense_csr(D)
    cycles = 3
    rb = bicg_residuals(D, b, cycles * ell)
    gammas = []
    errs = []

    def trace(cycle, rhat, uhat, r_new, y_new):
        v = rb[cycle * ell]
        for g in gammas:  # polynomials in D commute
            w, acc = v.copy(), v.copy()
            for j in range(ell):
                w = D @ w
                acc = acc - g[j] * w
            v = acc
        errs.append(np.linalg.norm(rhat[0] - v) / np.linalg.norm(v))
        g, *_ = np.linalg.lstsq(np.column_stack(rhat[1:]), rhat[0] - r_new, rcond=None)
        gammas.append(g)

    bicgstab_l(A, b, ell=ell, tol=1e-30, maxcycles=cycles, trace=trace)
    assert len(errs) == cycles and max(errs) <= 1e-8, errs


def test_one_cycle_when_l_reaches_the_distinct_eigenvalues():
    rng = np.random.default_rng(5)
    n = 40
    V = cn(rng, n, n) + 4 * np.eye(n)
    lam = np.array([2 + 1j, -1 + 0.5j, 3.0])[rng.integers(0, 3, n)]
    D = V @ np.diag(lam) @ np.linalg.inv(V)
    b = cn(rng, n)
    x, info = bicgstab_l(dense_csr(D), b, ell=3, tol=1e-10)
    assert info["status"] == O.OK and info["iterations"] == 1
    assert np.linalg.norm(D @ x - b) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("ell", [1, 4, 8])
def test_helmholtz_cube_matches_dense_lu(ell):
    A, b, _ = W.config_cube(7, seed=1)
    x, info = bicgstab_l(A, b, ell=ell, tol=1e-11)
    assert info["status"] == O.OK
    assert info["relres_true"] <= 1e-11 * (1 + 1e-2)
    xd = np.linalg.solve(O.to_dense(A), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_jacobi_equals_plain_method_on_scaled_matrix():
    A, b, _ = W.config_cylinder(h=0.25)
    diag = np.zeros(A.n, complex)
    rows = A.row_of_entry()
    on = A.col_idx == rows
    diag[rows[on]] = A.vals[on]
    S = CSR(A.row_ptr, A.col_idx, A.vals / diag[A.col_idx])  # A D^{-1}
    xj, ij = bicgstab_l(A, b, ell=4, tol=1e-30, maxcycles=5, jacobi=True)
    ys, iy = bicgstab_l(S, b, ell=4, tol=1e-30, maxcycles=5)
    assert np.linalg.norm(xj - ys / diag) <= 1e-11 * np.linalg.norm(xj)


def test_special_cases():
    A, b, _ = W.config_cube(5, seed=3)
    x, info = bicgstab_l(A, np.zeros(A.n, complex), ell=4)
    assert info["status"] == O.OK and info["iterations"] == 0 and not np.any(x)
    xd = np.linalg.solve(O.to_dense(A), b)
    x, info = bicgstab_l(A, b, ell=4, tol=1e-8, x0=xd)
    assert info["status"] == O.OK and info["iterations"] == 0
    x, info = bicgstab_l(A, b, ell=4, tol=1e-12, x0=0.5 * xd)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-12 * (1 + 1e-2)
