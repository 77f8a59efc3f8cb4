"""Pins of the reliable-update oracle (oracle/reliable.py), CPU only.

* Against the textbook solver written independently in C (oracle/krylov.c):
  run in double precision, with a reliable update whenever the residual has
  not grown since the last one, it must converge in the same number of
  iterations (within two) to the same solution.
* Against dense LAPACK: in complex64 it must reach the complex128 tolerance
  1e-10 (the true residual recomputed here with a dense product), which a
  complex64 iteration alone cannot, so at least two reliable updates happen;
  the error against the LU solution stays within the conditioning.
* Jacobi: the scaled iteration maps back through D^{-1} (a FEM system whose
  diagonal varies by orders of magnitude).
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.reliable import zbicgstab_reliable


def dense_relres(A, x, b):
    D = O.to_dense(A)
    return np.linalg.norm(b - D @ x) / np.linalg.norm(b)


def systems():
    A, b, _ = W.config_cube(6, k=9.0)
    yield "cube", A, b, False
    F, vals, rhs, ks, _ = W.config_freq_sweep(B=1, h=0.2, kmin=4.0, kmax=4.0, seed=3)
    yield "fem", F.with_vals(vals[0]), rhs[0], True


@pytest.mark.parametrize("case", ["cube", "fem"])
def test_double_precision_run_follows_the_textbook_solver(case):
    name, A, b, jacobi = next((s for s in systems() if s[0] == case))
    x_tb, i_tb = O.zbicgstab(A, b, tol=1e-10, jacobi=jacobi)
    x, info = zbicgstab_reliable(A, b, tol=1e-10, delta=1.0, jacobi=jacobi, inner=np.complex128)
    assert i_tb["status"] == 0 and info["status"] == 0
    assert abs(info["iterations"] - i_tb["iterations"]) <= 2, (info, i_tb)
    assert np.linalg.norm(x - x_tb) / np.linalg.norm(x_tb) < 1e-8


@pytest.mark.parametrize("case", ["cube", "fem"])
def test_complex64_iteration_reaches_the_double_tolerance(case):
    name, A, b, jacobi = next((s for s in systems() if s[0] == case))
    x, info = zbicgstab_reliable(A, b, tol=1e-10, delta=0.1, jacobi=jacobi, inner=np.complex64)
    assert info["status"] == 0, info
    assert info["outer_steps"] >= 2
    rr = dense_relres(A, x, b)
    assert rr <= 1e-10 * (1 + 1e-3)
    assert abs(rr - info["relres_true"]) <= 1e-3 * rr + 1e-16
    D = O.to_dense(A)
    xd = np.linalg.solve(D, b)
    kest = np.linalg.norm(D) * np.linalg.norm(xd) / np.linalg.norm(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= max(1e-8, 1e-9 * kest)


def test_without_updates_complex64_stalls_short_of_the_tolerance():
    """The updates are what carry the complex64 iteration past its own precision: with none (delta = 0, a
    flush only when the budget is spent) the true residual stays far above 1e-10."""
    A, b, _ = W.config_cube(6, k=9.0)
    x, info = zbicgstab_reliable(A, b, tol=1e-10, delta=0.0, maxiter=400, inner=np.complex64)
    assert info["status"] != 0
    assert dense_relres(A, x, b) > 1e-9


def test_zero_right_hand_side_and_breakdown_free_identity():
    A, b, _ = W.config_cube(4, k=9.0)
    x, info = zbicgstab_reliable(A, np.zeros(A.n, complex), tol=1e-10)
    assert info["status"] == 0 and info["iterations"] == 0 and not np.any(x)
    n = 50
    from workloads.csr import CSR

    I = CSR(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0 + 0j))
    rhs = np.arange(n) + 1j
    # in double precision the first step solves 2 I x = b exactly; in complex64 the first update leaves the
    # rounding of b / ||b|| (about 1e-8) and one more step removes it
    x, info = zbicgstab_reliable(I, rhs, tol=1e-10, jacobi=True, inner=np.complex128)
    assert info["status"] == 0 and info["iterations"] == 1
    assert np.allclose(x, rhs / 2, rtol=1e-14, atol=0)
    x, info = zbicgstab_reliable(I, rhs, tol=1e-10, jacobi=True)
    assert info["status"] == 0 and info["iterations"] <= 3 and info["outer_steps"] >= 2
    assert np.allclose(x, rhs / 2, rtol=1e-12, atol=0)
