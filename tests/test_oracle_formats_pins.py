"""Pins of the oracle's storage formats (ELL, HYB, SELL-C-sigma) against what their definitions fix.

- the 5 x 5 matrix of the paper's CSR illustration (Section 3.2) converted by
  hand to ELL, HYB of width 2, SELL-2-4 and SELL-2-1 with two lanes per row:
  every index and value written out below;
- converting back to CSR gives the original arrays bit for bit (ragged rows,
  empty rows, one long row, n not a multiple of C);
- products equal the CSR product: bit for bit where the row sums run in the
  same order (ELL, SELL, HYB with no COO part), to rounding otherwise;
- SELL ordering: lengths non-increasing inside each sigma window with ties in
  row order, sigma = 1 the identity, C = 1 with a global sort has no padding;
- HYB's default width from row-length histograms worked by hand.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import formats as F
from workloads.csr import CSR


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ragged(n=203, seed=0, maxlen=12):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen + 1, n)
    lens[[3, 50]] = 0
    lens[77] = 60
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(n, size=L, replace=False)) for L in lens]).astype(np.int32)
    return CSR(rp, ci, cn(rng, ci.size))


def same_csr(A, B):
    return (np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col_idx, B.col_idx)
            and np.array_equal(A.vals.view(np.float64), B.vals.view(np.float64)))


def test_paper_example_by_hand():
    A = W.csr_example()
    K, col, val, cr, cc, cv = F.to_ell(A)
    assert K == 3
    assert col.tolist() == [0, 1, 0, 1, 2, 1, 2, 2, 3, 4, -1, -1, -1, 4, -1]
    assert val.tolist() == [3, 8, 2, 4, 9, 14, 1, 6, 2, 7, 0, 0, 0, -1, 0]
    assert cr.size == 0
    K, col, val, cr, cc, cv = F.to_ell(A, 2)
    assert col.tolist() == [0, 1, 0, 1, 2, 1, 2, 2, 3, 4]
    assert val.tolist() == [3, 8, 2, 4, 9, 14, 1, 6, 2, 7]
    assert cr.tolist() == [3] and cc.tolist() == [4] and cv.tolist() == [-1]
    perm, ptr, col, val = F.to_sell(A, C=2, sigma=4)
    assert perm.tolist() == [3, 0, 1, 2, 4] and ptr.tolist() == [0, 6, 10, 14]
    assert col.tolist() == [1, 0, 3, 1, 4, -1, 1, 0, 2, 2, 2, -1, 4, -1]
    assert val.tolist() == [4, 3, 2, 14, -1, 0, 8, 2, 1, 6, 9, 0, 7, 0]
    perm, ptr, col, val = F.to_sell(A, C=2, sigma=1, t=2)
    assert perm.tolist() == [0, 1, 2, 3, 4] and ptr.tolist() == [0, 4, 12, 16]
    assert col.tolist() == [0, 1, 1, 2, 0, 2, 1, 3, -1, -1, 4, -1, 2, 4, -1, -1]
    assert val.tolist() == [3, 14, 8, 1, 2, 6, 4, 2, 0, 0, -1, 0, 9, 7, 0, 0]
    x = np.arange(1, 6) + 0.5j
    y = F.sell_spmv(5, 2, 2, perm, ptr, col, val, x)
    assert np.allclose(y, O.to_dense(A) @ x, rtol=1e-15, atol=0)


@pytest.mark.parametrize("K", [None, 0, 1, 5])
def test_ell_and_hyb_round_trip_and_product(K):
    A = ragged()
    x = cn(np.random.default_rng(4), A.n)
    Kk, col, val, cr, cc, cv = F.to_ell(A, K)
    lens = F.row_lengths(A)
    assert cr.size == int(np.maximum(lens - Kk, 0).sum())
    assert np.all(np.diff(cr) >= 0)
    assert same_csr(F.ell_to_csr(A.n, Kk, col, val, cr, cc, cv), A)
    y = F.ell_spmv(A.n, Kk, col, val, cr, cc, cv, x)
    yo = O.zspmv(A, x)
    if cr.size == 0:
        assert np.array_equal(y.view(np.float64), yo.view(np.float64))
    else:
        assert np.linalg.norm(y - yo) <= 1e-14 * np.linalg.norm(yo)
        assert np.allclose(y, O.to_dense(A) @ x, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("C,sigma,t", [(1, 1, 1), (4, 1, 1), (4, 16, 2), (64, 64, 1), (64, 256, 4), (8, 208, 1)])
def test_sell_round_trip_product_and_order(C, sigma, t):
    A = ragged()
    x = cn(np.random.default_rng(5), A.n)
    perm, ptr, col, val = F.to_sell(A, C, sigma, t)
    lens = F.row_lengths(A)
    assert sorted(perm.tolist()) == list(range(A.n))
    for w0 in range(0, A.n, sigma):
        win = perm[w0:w0 + sigma]
        assert sorted(win.tolist()) == list(range(w0, min(A.n, w0 + sigma)))
        L = lens[win]
        assert np.all(np.diff(L) <= 0)
        assert all(win[j] < win[j + 1] for j in range(len(win) - 1) if L[j] == L[j + 1])
    nch = -(-A.n // C)
    for c in range(nch):
        w = (ptr[c + 1] - ptr[c]) // C
        assert (ptr[c + 1] - ptr[c]) % C == 0 and w % t == 0
        assert w == -(-int(lens[perm[c * C:(c + 1) * C]].max()) // t) * t
    assert np.count_nonzero(col >= 0) == A.nnz and np.all(val[col < 0] == 0)
    assert same_csr(F.sell_to_csr(A.n, C, t, perm, ptr, col, val), A)
    y = F.sell_spmv(A.n, C, t, perm, ptr, col, val, x)
    assert np.array_equal(y.view(np.float64), O.zspmv(A, x).view(np.float64))


def test_sell_special_orders():
    A = ragged()
    perm, ptr, _, _ = F.to_sell(A, 16, 1)
    assert np.array_equal(perm, np.arange(A.n))
    perm, ptr, _, _ = F.to_sell(A, 1, A.n)
    assert ptr[-1] == A.nnz  # one row per chunk, no padding
    assert np.all(np.diff(F.row_lengths(A)[perm]) <= 0)


def test_hyb_default_width_by_hand():
    def mat(lens):
        n = len(lens)
        rp = np.zeros(n + 1, dtype=np.int32)
        rp[1:] = np.cumsum(lens)
        ci = np.concatenate([np.arange(L) % n for L in lens] + [np.zeros(0)]).astype(np.int32)
        return CSR(rp, ci, np.ones(ci.size, complex))

    assert F.hyb_default_width(mat([5, 5, 5, 1, 1, 1, 1, 1, 1])) == 5  # 3 of 9 rows have >= 5
    assert F.hyb_default_width(mat([5, 5, 4, 1, 1, 1, 1, 1, 1])) == 4
    assert F.hyb_default_width(mat([3, 2, 1])) == 3  # one row suffices when n = 3
    assert F.hyb_default_width(mat([2, 9, 2, 2])) == 2  # ceil(4/3) = 2 rows needed
    assert F.hyb_default_width(mat([0, 0, 0])) == 0
