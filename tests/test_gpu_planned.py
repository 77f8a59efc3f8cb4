"""The planned product in the caller's numbering (csr_zspmv_plan / csr_zspmv_planned) against the oracle.

The plan renumbers by level sets and keeps P A P^T; the product gathers P x, multiplies, and writes row k
of the result to y[perm[k]].  Each y_i is the same row sum as the plain product's, in another entry order
(the columns of a row are sorted in the new numbering), so the bound is the per-row one of the plain
product: |y_i - y_oracle_i| <= 16 eps sum_j |a_ij| |x_j|, plus 1e-14 normwise.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from workloads.csr import CSR, permute_symmetric

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def cn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def check(A, y, x):
    yo = O.zspmv(A, x)
    rows = O.zspmv(A.with_vals(np.abs(A.vals).astype(np.complex128)), np.abs(x).astype(np.complex128)).real
    assert np.all(np.abs(y - yo) <= 16 * EPS * rows + 1e-300)
    if np.linalg.norm(yo) > 0:
        assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= 1e-14


def ragged(n=3001, seed=0, maxlen=16):
    """Rows of 0..maxlen entries (empty rows at 5, 17 and the last), one 600-entry row, symmetric pattern not
    required; columns sorted within rows."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen + 1, size=n)
    lens[[5, 17, n - 1]] = 0
    lens[100] = 600
    cols = [np.sort(rng.choice(n, size=int(k), replace=False)) for k in lens]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(lens, out=rp[1:])
    ci = np.concatenate(cols).astype(np.int32)
    return CSR(rp, ci, cn(rng, ci.size))


@pytest.mark.parametrize("case", ["scrambled_cube", "ragged", "scrambled_cylinder"])
def test_planned_product_matches_the_oracle(hz, case):
    if case == "scrambled_cube":
        A, _, _ = W.config_cube(16, seed=2)
        A = permute_symmetric(A, np.random.default_rng(4).permutation(A.n))
    elif case == "ragged":
        A = ragged()
    else:
        A, _, _ = W.config_cylinder(h=0.08)
        A = permute_symmetric(A, np.random.default_rng(5).permutation(A.n))
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    plan = hz.csr_zspmv_plan(rp, ci, v)
    rng = np.random.default_rng(9)
    for _ in range(2):  # the plan is reused
        x = cn(rng, A.n)
        y = hz.csr_zspmv_planned(plan, dev(x)).cpu().numpy()
        check(A, y, x)
    if case == "ragged":
        assert np.all(y[[5, 17, A.n - 1]] == 0)


def test_full_size_cabin_in_its_random_numbering(hz):
    A, _, _ = W.config_cabin()
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    plan = hz.csr_zspmv_plan(rp, ci, v)
    x = cn(np.random.default_rng(3), A.n)
    y = hz.csr_zspmv_planned(plan, dev(x)).cpu().numpy()
    check(A, y, x)


def test_rebuild_after_new_values_empty_matrix_and_invalid_arguments(hz):
    A, _, _ = W.config_cube(8, seed=1)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    plan = hz.csr_zspmv_plan(rp, ci, v)
    x = cn(np.random.default_rng(1), A.n)
    vals2 = A.vals * (0.5 - 2j)
    v.copy_(dev(vals2))
    y_old = hz.csr_zspmv_planned(plan, dev(x)).cpu().numpy()
    check(A, y_old, x)  # the plan keeps the values it was built with
    plan = hz.csr_zspmv_plan(rp, ci, v)
    check(A.with_vals(vals2), hz.csr_zspmv_planned(plan, dev(x)).cpu().numpy(), x)
    # a matrix with no entries: y = 0
    n = 50
    E = CSR(np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.complex128))
    pe = hz.csr_zspmv_plan(dev(E.row_ptr), dev(E.col_idx), dev(E.vals))
    ye = hz.csr_zspmv_planned(pe, dev(np.ones(n, complex)), torch.full((n,), 3.0 + 0j, dtype=torch.complex128, device="cuda:0"))
    assert torch.count_nonzero(ye).item() == 0
    # x and y overlapping, a plan too small
    xx = dev(x)
    with pytest.raises(hz.HelmzError):
        hz.csr_zspmv_planned(plan, xx, xx)
    small = {"n": plan["n"], "nnz": plan["nnz"], "plan": plan["plan"][:1024]}
    with pytest.raises((hz.HelmzError, ValueError)):
        hz.csr_zspmv_planned(small, xx)
