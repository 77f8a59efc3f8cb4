"""GPU parity of the storage formats (ELL / HYB, SELL-C-sigma) against the oracle.

Conversions are index and byte work: the GPU's arrays (permutation, chunk
pointers, columns, values, COO triplets) must equal the oracle's bit for bit.
Products are floating point: every y_i within 16 eps (|A| |x|)_i of the
oracle's CSR product (the GPU fuses multiply-adds and, with t > 1 lanes per
row, sums a row in another order).
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import formats as F
from workloads.csr import CSR

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ragged(n=2003, seed=0, maxlen=40):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen + 1, n)
    lens[[5, 17, n - 1]] = 0
    lens[100] = min(600, n)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(n, size=L, replace=False)) for L in lens]).astype(np.int32)
    return CSR(rp, ci, cn(rng, ci.size))


def dcsr(A):
    return dev(A.row_ptr), dev(A.col_idx), dev(A.vals)


def check_y(A, x, y):
    yo = O.zspmv(A, x)
    bound = 16 * EPS * O.zspmv(A.with_vals(np.abs(A.vals).astype(complex)), np.abs(x).astype(complex)).real
    assert np.all(np.abs(y - yo) <= bound + 1e-300), np.max(np.abs(y - yo) / (bound + 1e-300))


def same(a, b):
    a = a.cpu().numpy() if isinstance(a, torch.Tensor) else a
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def check_hyb(hz, A, K):
    rp, ci, v = dcsr(A)
    h = hz.csr_to_hyb(rp, ci, v, K=K)
    Ko, col, val, cr, cc, cv = F.to_ell(A, None if K == "ell" else (F.hyb_default_width(A) if K is None else K))
    assert h["K"] == Ko
    assert same(h["ell_col"], col) and same(h["ell_val"], val)
    assert same(h["coo_row"], cr) and same(h["coo_col"], cc) and same(h["coo_val"], cv)
    x = cn(np.random.default_rng(7), A.n)
    y = hz.hyb_zspmv(h, dev(x)).cpu().numpy()
    check_y(A, x, y)
    return h


def check_sell(hz, A, C, sigma, t):
    rp, ci, v = dcsr(A)
    s = hz.csr_to_sell(rp, ci, v, C=C, sigma=sigma, t=t)
    perm, ptr, col, val = F.to_sell(A, C, sigma, t)
    assert same(s["perm"], perm) and same(s["chunk_ptr"], ptr)
    assert same(s["col"], col) and same(s["val"], val)
    x = cn(np.random.default_rng(8), A.n)
    y = hz.sell_zspmv(s, dev(x)).cpu().numpy()
    check_y(A, x, y)
    return s


def test_paper_example(hz):
    A = W.csr_example()
    assert hz.csr_row_stats(dev(A.row_ptr)) == (3, 2)
    check_hyb(hz, A, "ell")
    check_hyb(hz, A, 2)
    check_sell(hz, A, 2, 4, 1)
    check_sell(hz, A, 2, 1, 2)


@pytest.mark.parametrize("K", [None, "ell", 0, 1, 7])
def test_hyb_ragged(hz, K):
    A = ragged()
    mx, Kd = hz.csr_row_stats(dev(A.row_ptr))
    assert mx == int(F.row_lengths(A).max()) and Kd == F.hyb_default_width(A)
    check_hyb(hz, A, K)


@pytest.mark.parametrize("C,sigma,t", [(64, 1, 1), (64, 2048, 1), (64, 64, 2), (32, 256, 4), (7, 700, 8), (1, 1, 1),
                                       (1024, 1024, 2)])
def test_sell_ragged(hz, C, sigma, t):
    check_sell(hz, ragged(), C, sigma, t)


@pytest.mark.parametrize("t", [1, 2])
def test_cylinder_small(hz, t):
    A, _, _ = W.config_cylinder(h=0.1)
    check_sell(hz, A, 64, 2048, t)
    check_hyb(hz, A, None)


def test_full_size_cylinder(hz):
    A, _, _ = W.config_cylinder()
    assert A.n == 209777
    rp, ci, v = dcsr(A)
    x = cn(np.random.default_rng(9), A.n)
    xd = dev(x)
    s = hz.csr_to_sell(rp, ci, v, C=64, sigma=2048, t=1)
    perm = F.sell_perm(A, 2048)
    assert same(s["perm"], perm)
    assert int(s["chunk_ptr"][-1]) == s["col"].numel() and int((s["col"] >= 0).sum()) == A.nnz
    check_y(A, x, hz.sell_zspmv(s, xd).cpu().numpy())
    h = hz.csr_to_hyb(rp, ci, v)
    assert h["coo_row"].numel() == int(np.maximum(F.row_lengths(A) - h["K"], 0).sum())
    check_y(A, x, hz.hyb_zspmv(h, xd).cpu().numpy())


def test_edge_cases_and_invalid_arguments(hz):
    one = CSR(np.array([0, 0], dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0, complex))
    s = hz.csr_to_sell(*dcsr(one), C=64, sigma=64)
    assert s["col"].numel() == 0 and s["chunk_ptr"].cpu().tolist() == [0, 0]
    assert hz.sell_zspmv(s, dev(np.array([1 + 1j]))).cpu().tolist() == [0j]
    h = hz.csr_to_hyb(*dcsr(one))
    assert h["K"] == 0 and hz.hyb_zspmv(h, dev(np.array([2j]))).cpu().tolist() == [0j]
    A = ragged(n=300, seed=3)
    rp, ci, v = dcsr(A)
    for bad in (dict(C=0), dict(C=2000), dict(t=3), dict(C=64, sigma=100)):
        with pytest.raises(hz.HelmzError):
            hz.csr_to_sell(rp, ci, v, **bad)
    broken = ci.clone()
    broken[3] = A.n  # a column out of range: rejected by the conversions' validation
    with pytest.raises(hz.HelmzError):
        hz.csr_to_sell(rp, broken, v)
    with pytest.raises(hz.HelmzError):
        hz.csr_to_hyb(rp, broken, v)
