"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

None of these compares the oracle with itself: expected values come from the
paper's worked CSR example, hand-worked small-integer arithmetic, closed
forms, LAPACK dense solves, a discrete plane wave and finite differences.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.csr import CSR


def _example(g):
    ia = g["ia_1based"].astype(np.int32) - 1
    ja = g["ja_1based"].astype(np.int32) - 1
    return CSR(ia, ja, g["aa"].astype(np.complex128))


# ---------------------------------------------------------------- SpMV (Section 3.2)


def test_csr_example_layout(golden_csr_example):
    g = golden_csr_example
    A = _example(g)
    assert A.row_ptr[-1] == A.nnz == 11
    assert g["ia_1based"][-1] == A.nnz + 1  # IA(n+1) = nz + 1
    D = O.to_dense(A).real
    assert np.array_equal(D, g["matrix"])


def test_csr_example_spmv_exact(golden_csr_example):
    g = golden_csr_example
    A = _example(g)
    assert np.array_equal(O.zspmv(A, g["x_ones"]), g["y_ones"])
    assert np.array_equal(O.zspmv(A, g["x_ramp"]), g["y_ramp"])
    # complexified: values scaled by (1+2i) scale the product exactly
    Ac = A.with_vals(A.vals * (1 + 2j))
    assert np.array_equal(O.zspmv(Ac, g["x_ramp"]), (1 + 2j) * g["y_ramp"])
    # complex x: A (i * ramp) = i * y
    assert np.array_equal(O.zspmv(A, 1j * g["x_ramp"]), 1j * g["y_ramp"])


def test_spmv_complex_small_integers():
    # [[1+i, 2], [0, 3-2i]] @ [2-i, 1+4i] worked by hand:
    # row0 = (1+i)(2-i) + 2(1+4i) = (3+i) + (2+8i) = 5+9i
    # row1 = (3-2i)(1+4i) = 3 + 12i - 2i + 8 = 11+10i
    A = CSR(np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32), np.array([1 + 1j, 2, 3 - 2j]))
    assert np.array_equal(O.zspmv(A, np.array([2 - 1j, 1 + 4j])), np.array([5 + 9j, 11 + 10j]))


def test_complex64_spmv_small_integers():
    A = CSR(np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32), np.array([1 + 1j, 2, 3 - 2j]))
    y = O.cspmv(A, np.array([2 - 1j, 1 + 4j]))
    assert y.dtype == np.complex64
    assert np.array_equal(y, np.array([5 + 9j, 11 + 10j], dtype=np.complex64))


# ---------------------------------------------------------------- BLAS-1 (Section 5)


def test_zdotc_small_integers_conjugates_first_argument():
    x = np.array([1 + 2j, 3 - 1j])
    y = np.array([2 - 1j, 1 + 4j])
    # conj(x).y = (1-2i)(2-i) + (3+i)(1+4i) = (-5i) + (-1+13i) = -1+8i
    assert O.zdotc(x, y) == -1 + 8j
    assert O.zdotc(y, x) == -1 - 8j


def test_zdotc_closed_forms():
    n = 1000
    rng = np.random.default_rng(3)
    theta = rng.uniform(0, 2 * np.pi, n)
    x = np.exp(1j * theta)
    assert abs(O.zdotc(x, x) - n) < 1e-12 * n
    phi = 0.37
    z = np.exp(1j * phi)
    powers = z ** np.arange(n)
    geo = (1 - z**n) / (1 - z)
    assert abs(O.zdotc(np.ones(n), powers) - geo) < 1e-11 * n
    assert abs(O.zdotc(powers, np.ones(n)) - np.conj(geo)) < 1e-11 * n


def test_nrm2_closed_forms():
    assert O.dznrm2(np.array([3 + 4j, 0j])) == 5.0
    assert O.dznrm2(np.array([1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j])) == np.sqrt(8.0)
    n = 4096
    x = np.exp(1j * np.linspace(0, 5, n))
    assert abs(O.dznrm2(x) - 64.0) < 1e-12


def test_zaxpy_scal_xmy_exact():
    alpha = 2 - 1j
    x = np.array([1 + 1j, -3 + 0j])
    y = np.array([4 + 0j, 2j])
    # (2-i)(1+i)+4 = 7+i ; (2-i)(-3)+2i = -6+5i
    assert np.array_equal(O.zaxpy(alpha, x, y), np.array([7 + 1j, -6 + 5j]))
    assert np.array_equal(O.zscal(alpha, x), np.array([3 + 1j, -6 + 3j]))
    assert np.array_equal(O.zxmy(x, y), np.array([4 + 4j, -6j]))


# ---------------------------------------------------------------- generators (stencil) and plane wave


def test_plane_wave_annihilated_by_interior_rows():
    N = 20
    A, _, _ = W.config_cube(N)
    h, k = A.meta["h"], A.meta["k"]
    kappa = (2.0 / h) * np.arcsin(k * h / 2.0)
    u = W.plane_wave(A.meta["coords"], kappa, axis=0)
    Au = O.zspmv(A, u)
    interior = A.meta["interior_rows"]
    boundary = A.meta["boundary_rows"]
    assert np.max(np.abs(Au[interior])) < 1e-13
    assert np.max(np.abs(Au[boundary])) > 0.1
    # with the continuous wavenumber the interior residual is not zero
    Au_k = O.zspmv(A, W.plane_wave(A.meta["coords"], k, axis=0))
    assert np.max(np.abs(Au_k[interior])) > 1e-3


def test_plane_wave_recovered_by_solver():
    A, _, _ = W.config_cube(10)
    h, k = A.meta["h"], A.meta["k"]
    kappa = (2.0 / h) * np.arcsin(k * h / 2.0)
    u = W.plane_wave(A.meta["coords"], kappa, axis=1)
    b = O.zspmv(A, u)
    x, info = O.zbicgstab(A, b, tol=1e-12)
    assert info["status"] == O.OK
    cond = np.linalg.cond(O.to_dense(A))
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 10 * cond * 1e-12


# ---------------------------------------------------------------- BiCGStab vs LAPACK (Section 7)


@pytest.mark.parametrize("jacobi", [False, True])
@pytest.mark.parametrize("N", [8, 10])
def test_bicgstab_matches_dense_lu_cube(N, jacobi):
    A, b, _ = W.config_cube(N, seed=N)
    tol = 1e-10
    x, info = O.zbicgstab(A, b, tol=tol, jacobi=jacobi)
    assert info["status"] == O.OK
    assert info["relres_true"] <= 2 * tol
    xd = O.dense_solve(A, b)
    cond = np.linalg.cond(O.to_dense(A))
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * cond * tol
    # independent residual check with numpy
    D = O.to_dense(A)
    assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 2 * tol


@pytest.mark.parametrize("robin", ["all", "caps"])
def test_bicgstab_matches_dense_lu_small_cylinder(robin):
    A, b, _ = W.config_cylinder(h=1.0 / 3.0, k=3.0, seed=1, robin=robin)
    assert A.n <= 1000
    tol = 1e-10
    x, info = O.zbicgstab(A, b, tol=tol, jacobi=True)
    assert info["status"] == O.OK
    D = O.to_dense(A)
    assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 2 * tol
    xd = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * np.linalg.cond(D) * tol


def test_bicgstab_half_step_exit_scaled_identity():
    n = 7
    alpha = 2.5 - 0.5j
    A = CSR(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, alpha))
    b = np.arange(1, n + 1) * (1 + 1j)
    x, info = O.zbicgstab(A, b, tol=1e-14)
    assert info["status"] == O.OK and info["iterations"] == 1
    assert np.allclose(x, b / alpha, rtol=1e-15, atol=0)


def test_bicgstab_jacobi_diagonal_one_step():
    n = 9
    d = (np.arange(n) + 1.0) * (1 - 0.25j)
    A = CSR(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.ones(n) + 2j
    x, info = O.zbicgstab(A, b, tol=1e-14, jacobi=True)
    assert info["status"] == O.OK and info["iterations"] == 1
    assert np.allclose(x, b / d, rtol=1e-14, atol=0)
    # without the preconditioner a spread-out diagonal needs more steps
    _, info2 = O.zbicgstab(A, b, tol=1e-14, jacobi=False)
    assert info2["iterations"] > 1


def test_bicgstab_zero_rhs():
    A, _, _ = W.config_cube(4)
    x, info = O.zbicgstab(A, np.zeros(A.n), tol=1e-8, x0=np.ones(A.n))
    assert info["status"] == O.OK and info["iterations"] == 0
    assert np.all(x == 0)


def test_bicgstab_breakdown_sigma_zero():
    # A = [[0,1],[1,0]], b = e1: v = A r = e2, <rhat, v> = <e1, e2> = 0
    A = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
    _, info = O.zbicgstab(A, np.array([1.0 + 0j, 0j]), tol=1e-8)
    assert info["status"] == O.BREAKDOWN and info["iterations"] == 1


def test_bicgstab_maxiter_and_nonfinite_and_invalid():
    A, b, _ = W.config_cube(8)
    _, info = O.zbicgstab(A, b, tol=1e-12, maxiter=1)
    assert info["status"] == O.NOT_CONVERGED and info["iterations"] == 1
    bn = b.copy()
    bn[3] = np.nan
    _, info = O.zbicgstab(A, bn, tol=1e-8)
    assert info["status"] == O.NONFINITE
    Z = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
    _, info = O.zbicgstab(Z, np.ones(2, complex), tol=1e-8, jacobi=True)
    assert info["status"] == O.INVALID


def test_complex64_solver_tracks_complex128():
    A, b, _ = W.config_cube(8, seed=2)
    x32, info32 = O.cbicgstab(A, b, tol=1e-5)
    x64, info64 = O.zbicgstab(A, b, tol=1e-12)
    assert info32["status"] == O.OK and x32.dtype == np.complex64
    D = O.to_dense(A)
    r = np.linalg.norm(b - D @ x32.astype(np.complex128)) / np.linalg.norm(b)
    assert r < 1e-4
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-3


# ---------------------------------------------------------------- mixed-precision refinement


def test_mixed_refinement_reaches_fp64_tolerance():
    A, b, _ = W.config_cube(10, seed=4)
    x, info = O.zbicgstab_mixed(A, b, tol=1e-10, inner_tol=1e-4)
    assert info["status"] == O.OK
    assert info["outer_steps"] >= 2  # one complex64 solve alone cannot reach 1e-10
    D = O.to_dense(A)
    assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-10
    xd = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 10 * np.linalg.cond(D) * 1e-10


# ---------------------------------------------------------------- adjoint / gradients


def _loss(x, rec, t):
    return float(np.sum(np.abs(x[rec] - t) ** 2))


def _grad_x(x, rec, t):
    # real-pair gradient of sum |x_r - t_r|^2: 2 (x_r - t_r)
    g = np.zeros_like(x)
    g[rec] = 2.0 * (x[rec] - t)
    return g


def test_conj_transpose_and_lambda_match_dense():
    A, b, _ = W.config_cube(6, seed=5)
    A = A.with_vals(A.vals + 0.3j * np.sin(np.arange(A.nnz)))  # make A non-symmetric
    D = O.to_dense(A)
    AH = O.zcsr_conj_transpose(A)
    assert np.array_equal(O.to_dense(AH), D.conj().T)
    rng = np.random.default_rng(0)
    g = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    x = np.linalg.solve(D, b)
    lam, gv, info = O.zadjoint(A, x, g, tol=1e-12)
    lam_d = np.linalg.solve(D.conj().T, g)
    assert np.linalg.norm(lam - lam_d) / np.linalg.norm(lam_d) < 1e-8
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.allclose(gv, -lam_d[rows] * np.conj(x[A.col_idx]), rtol=1e-7, atol=1e-12)


def test_linear_functional_gradient_closed_form():
    # L = Re(c^H x) has real-pair gradient c wrt x, so grad_b = A^{-H} c.
    A, b, _ = W.config_cube(6, seed=6)
    D = O.to_dense(A)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    x = np.linalg.solve(D, b)
    lam, _, _ = O.zadjoint(A, x, c, tol=1e-12)
    eps = 1e-6
    for j in (0, 17, 100):
        e = np.zeros(A.n, complex)
        e[j] = 1.0
        Lp = np.real(np.vdot(c, np.linalg.solve(D, b + eps * e)))
        Lm = np.real(np.vdot(c, np.linalg.solve(D, b - eps * e)))
        Lpi = np.real(np.vdot(c, np.linalg.solve(D, b + 1j * eps * e)))
        Lmi = np.real(np.vdot(c, np.linalg.solve(D, b - 1j * eps * e)))
        fd = (Lp - Lm) / (2 * eps) + 1j * (Lpi - Lmi) / (2 * eps)
        assert abs(fd - lam[j]) < 1e-6 * max(1.0, abs(lam[j]))


def test_entry_gradient_matches_central_differences():
    A, b, _ = W.config_cube(5, seed=7)
    D = O.to_dense(A)
    rng = np.random.default_rng(2)
    rec = rng.choice(A.n, 20, replace=False)
    t = rng.standard_normal(20) + 1j * rng.standard_normal(20)
    x = np.linalg.solve(D, b)
    lam, gv, _ = O.zadjoint(A, x, _grad_x(x, rec, t), tol=1e-13)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    for p in rng.choice(A.nnz, 12, replace=False):
        i, j = rows[p], A.col_idx[p]
        eps = 1e-6
        vals = []
        for d in (eps, -eps, 1j * eps, -1j * eps):
            Dp = D.copy()
            Dp[i, j] += d
            vals.append(_loss(np.linalg.solve(Dp, b), rec, t))
        fd = (vals[0] - vals[1]) / (2 * eps) + 1j * (vals[2] - vals[3]) / (2 * eps)
        assert abs(fd - gv[p]) <= 1e-5 * max(1e-3, abs(gv[p])), (p, fd, gv[p])


def test_bicgstab_first_step_defining_properties():
    """One BiCGStab step from x0 = 0 (no preconditioner): with rhat = r0 = b and p = b,
    alpha makes s = b - alpha A b orthogonal to rhat (the bi-orthogonality condition) and
    omega minimises ||s - omega t|| (t = A s), so r1 = s - omega t is orthogonal to t.
    x1 = alpha b + omega s is then the oracle's iterate after maxiter = 1."""
    rng = np.random.default_rng(12)
    n = 6
    D = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    rows, cols = np.nonzero(np.ones((n, n)))
    A = CSR(np.arange(0, n * n + 1, n, dtype=np.int32), cols.astype(np.int32), D[rows, cols].astype(complex))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x1, info = O.zbicgstab(A, b, tol=1e-15, maxiter=1)
    assert info["status"] == O.NOT_CONVERGED and info["iterations"] == 1
    r1 = b - D @ x1
    # the iterate lies in span{b, A b}; recover alpha and omega from it without the oracle's formulas
    Ab = D @ b
    # x1 = alpha b + omega (b - alpha A b) = (alpha + omega) b - alpha omega A b
    coef, *_ = np.linalg.lstsq(np.stack([b, Ab], axis=1), x1, rcond=None)
    assert np.linalg.norm(np.stack([b, Ab], axis=1) @ coef - x1) <= 1e-12 * np.linalg.norm(x1)
    # alpha from the bi-orthogonality condition <b, b - alpha A b> = 0
    alpha = np.vdot(b, b) / np.vdot(b, Ab)
    s = b - alpha * Ab
    assert abs(np.vdot(b, s)) <= 1e-12 * np.linalg.norm(b) * np.linalg.norm(s)
    t = D @ s
    assert abs(np.vdot(t, r1)) <= 1e-12 * np.linalg.norm(t) * np.linalg.norm(r1)
    # and r1 is the least-squares residual of s on t
    w_ls = np.vdot(t, s) / np.vdot(t, t)
    assert np.linalg.norm(r1 - (s - w_ls * t)) <= 1e-12 * np.linalg.norm(s)
