"""The threaded oracle build (timing only) against the sequential oracle.

The threaded build splits rows and element-wise loops across threads, which
changes no result, and sums dot products per thread, which changes only
their rounding order.  So its product must equal the sequential product bit
for bit, and its BiCGStab must reach the same tolerance with an iteration
count within a few percent.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W



def test_threaded_product_is_bitwise_sequential():
    A, _, _ = W.config_cylinder(h=0.1)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    assert np.array_equal(O.zspmv_omp(A, x).view(np.float64), O.zspmv(A, x).view(np.float64))


@pytest.mark.parametrize("jacobi", [False, True])
def test_threaded_solve_matches_sequential(jacobi):
    A, b, _ = W.config_cube(12, seed=3)
    xs, i_s = O.zbicgstab(A, b, tol=1e-10, jacobi=jacobi)
    xt, i_t = O.zbicgstab_omp(A, b, tol=1e-10, jacobi=jacobi)
    assert i_s["status"] == O.OK and i_t["status"] == O.OK
    assert abs(i_t["iterations"] - i_s["iterations"]) <= max(2, i_s["iterations"] // 20)
    rr = np.linalg.norm(b - O.zspmv(A, xt)) / np.linalg.norm(b)
    assert rr <= 1e-10 * 1.01
    assert O.omp_threads() >= 1
