"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Every input is seeded and synthetic.  Floating-point comparisons use bounds
derived from the arithmetic:
  - SpMV, per row: |y - y_oracle| <= 16 eps (|A| |x|)_row, and normwise
    ||y - y_oracle|| / ||y_oracle|| <= 1e-14 on the workloads;
  - dot products: |d - d_oracle| <= n eps sum |x_i| |y_i|;
  - solves: the true residual of the GPU solution, recomputed with the
    oracle's SpMV, meets the requested tolerance.
"""

import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from workloads.csr import CSR

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def dev_csr(A, vdtype=torch.complex128):
    return dev(A.row_ptr), dev(A.col_idx), dev(A.vals, vdtype)


def cn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def ragged_matrix(n=3001, seed=0, maxlen=40):
    """Random row lengths 0..maxlen, a few empty rows, one row of 600 entries."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen + 1, n)
    lens[[5, 17, n - 1]] = 0
    lens[100] = min(600, n)
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = np.sort(rng.choice(n, size=L, replace=False))
        rows.append(np.full(L, i))
        cols.append(c)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(lens, out=rp[1:])
    ci = np.concatenate(cols).astype(np.int32)
    return CSR(rp, ci, cn(rng, ci.size))


def abs_rowsum(A, x):
    return O.zspmv(A.with_vals(np.abs(A.vals).astype(np.complex128)), np.abs(x).astype(np.complex128)).real


def check_spmv(hz, A, x, rtol_rows=16 * EPS, rtol_norm=1e-14):
    rp, ci, v = dev_csr(A)
    y = hz.csr_zspmv(rp, ci, v, dev(x)).cpu().numpy()
    yo = O.zspmv(A, x)
    bound = rtol_rows * abs_rowsum(A, x) + 1e-300
    assert np.all(np.abs(y - yo) <= bound), np.max(np.abs(y - yo) / bound)
    if np.linalg.norm(yo) > 0:
        assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= rtol_norm
    return y


# ---------------------------------------------------------------- SpMV


def test_spmv_paper_example_exact(hz, golden_csr_example):
    g = golden_csr_example
    A = CSR(g["ia_1based"].astype(np.int32) - 1, g["ja_1based"].astype(np.int32) - 1, g["aa"].astype(complex))
    rp, ci, v = dev_csr(A)
    assert np.array_equal(hz.csr_zspmv(rp, ci, v, dev(g["x_ones"].astype(complex))).cpu().numpy(), g["y_ones"])
    assert np.array_equal(hz.csr_zspmv(rp, ci, v, dev(g["x_ramp"].astype(complex))).cpu().numpy(), g["y_ramp"])
    vc = dev(A.vals * (1 + 2j))
    yc = hz.csr_zspmv(rp, ci, vc, dev(g["x_ramp"].astype(complex))).cpu().numpy()
    assert np.array_equal(yc, (1 + 2j) * g["y_ramp"])


@pytest.mark.parametrize("lanes", [2, 4, 8, 16, 32, 64])
def test_spmv_every_lane_width_ragged(hz, lanes, monkeypatch):
    monkeypatch.setenv("HZ_SPMV_LANES", str(lanes))
    A = ragged_matrix(seed=lanes)
    x = cn(np.random.default_rng(1), A.n)
    y = check_spmv(hz, A, x)
    assert np.all(y[[5, 17, A.n - 1]] == 0)


@pytest.mark.parametrize("form", ["rows", "tiles"])
@pytest.mark.parametrize("maxlen", [3, 16, 40])
def test_spmv_both_forms_ragged(hz, form, maxlen, monkeypatch):
    """Both standalone forms on ragged rows: tiles that fit the LDS buffer
    (short rows), tiles that do not (long rows: the vector fallback), a
    600-entry row, empty rows, a ragged last tile (n = 3001)."""
    monkeypatch.setenv("HZ_SPMV_FORM", form)
    A = ragged_matrix(seed=maxlen, maxlen=maxlen)
    x = cn(np.random.default_rng(7), A.n)
    y = check_spmv(hz, A, x)
    assert np.all(y[[5, 17, A.n - 1]] == 0)
    rp, ci, v = dev_csr(A)
    y2 = hz.csr_zspmv(rp, ci, v, dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.float64), y2.view(np.float64))


def test_spmv_tiles_with_blocks_looping_over_tiles(hz, monkeypatch):
    """The tile form above 4,096 tiles, where 1,024 blocks loop over the tiles
    and hold their results in LDS for several tiles before storing them: a
    tile count that is no multiple of the hold depth, a ragged last tile,
    empty rows and rows too long for the LDS buffer among the short ones."""
    monkeypatch.setenv("HZ_SPMV_FORM", "tiles")
    n = 64 * 4133 + 29
    rng = np.random.default_rng(41)
    lens = rng.integers(0, 13, n)
    lens[[3, 64 * 2000, n - 1]] = 0
    lens[[70, 64 * 3001 + 5]] = [600, 900]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(lens, out=rp[1:])
    ci = rng.integers(0, n, rp[-1]).astype(np.int32)
    A = CSR(rp, ci, cn(rng, ci.size))
    x = cn(np.random.default_rng(42), n)
    y = check_spmv(hz, A, x)
    assert np.all(y[[3, 64 * 2000, n - 1]] == 0)


@pytest.mark.parametrize("form", ["rows", "tiles"])
def test_spmv_both_forms_complex64_and_rect(hz, form, monkeypatch):
    monkeypatch.setenv("HZ_SPMV_FORM", form)
    A = ragged_matrix(n=2000, seed=3, maxlen=20)
    x = cn(np.random.default_rng(8), A.n).astype(np.complex64)
    rp, ci, v = dev_csr(A, torch.complex64)
    y = hz.csr_cspmv(rp, ci, v, dev(x)).cpu().numpy()
    bound = 32 * EPS32 * abs_rowsum(A, x.astype(np.complex128))
    assert np.all(np.abs(y.astype(complex) - O.cspmv(A, x).astype(complex)) <= bound)
    # rectangular: the first 700 rows of A restricted to columns < 1500
    keep = A.col_idx < 1500
    rows = A.row_of_entry()
    sel = keep & (rows < 700)
    rpr = np.zeros(701, np.int32)
    np.cumsum(np.bincount(rows[sel], minlength=700), out=rpr[1:])
    R = CSR(rpr, A.col_idx[sel], A.vals[sel])
    xr = cn(np.random.default_rng(9), 1500)
    yr = hz.csr_zspmv_rect(dev(R.row_ptr), dev(R.col_idx), dev(R.vals), dev(xr)).cpu().numpy()
    Rd = np.zeros((700, 1500), complex)
    Rd[R.row_of_entry(), R.col_idx] = R.vals
    assert np.allclose(yr, Rd @ xr, rtol=0, atol=1e-13 * np.abs(Rd).sum(1).max() * np.abs(xr).max())


@pytest.mark.parametrize("lanes", [2, 8, 16, 64])
def test_spmv_every_lane_width_cube(hz, lanes, monkeypatch):
    monkeypatch.setenv("HZ_SPMV_LANES", str(lanes))
    A, _, _ = W.config_cube(12)
    check_spmv(hz, A, cn(np.random.default_rng(2), A.n))


@pytest.mark.parametrize("n", [1, 2, 7, 64, 255, 257, 4097])
def test_spmv_small_and_ragged_sizes(hz, n):
    A = ragged_matrix(n=max(n, 101), seed=n) if n > 100 else None
    if A is None:
        rng = np.random.default_rng(n)
        lens = rng.integers(1, 5, n)
        rp = np.zeros(n + 1, np.int32)
        np.cumsum(lens, out=rp[1:])
        ci = rng.integers(0, n, rp[-1]).astype(np.int32)
        A = CSR(rp, ci, cn(rng, rp[-1]))
    check_spmv(hz, A, cn(np.random.default_rng(3), A.n))


def test_spmv_cube_workload(hz):
    A, b, _ = W.config_cube(20)
    check_spmv(hz, A, cn(np.random.default_rng(0), A.n))


def test_spmv_cylinder_workload_full_size(hz):
    A, b, _ = W.config_cylinder()
    assert A.n == 209777
    check_spmv(hz, A, cn(np.random.default_rng(0), A.n))


def test_spmv_cabin_workload_full_size(hz):
    A, b, _ = W.config_cabin()
    assert A.n > 1_000_000
    check_spmv(hz, A, cn(np.random.default_rng(0), A.n))


def test_spmv_deterministic(hz):
    A, _, _ = W.config_cylinder(h=0.08)
    rp, ci, v = dev_csr(A)
    x = dev(cn(np.random.default_rng(5), A.n))
    y1 = hz.csr_zspmv(rp, ci, v, x).cpu().numpy()
    y2 = hz.csr_zspmv(rp, ci, v, x).cpu().numpy()
    assert np.array_equal(y1.view(np.float64), y2.view(np.float64))


def test_cspmv_parity(hz):
    A, _, _ = W.config_cylinder(h=0.08)
    x = cn(np.random.default_rng(6), A.n).astype(np.complex64)
    rp, ci, v = dev_csr(A, torch.complex64)
    y = hz.csr_cspmv(rp, ci, v, dev(x)).cpu().numpy()
    assert y.dtype == np.complex64
    yo = O.cspmv(A, x)
    bound = 32 * EPS32 * abs_rowsum(A, x.astype(np.complex128))
    assert np.all(np.abs(y.astype(complex) - yo.astype(complex)) <= bound)


def test_spmv_rejects_aliasing_and_bad_sizes(hz):
    A, _, _ = W.config_cube(4)
    rp, ci, v = dev_csr(A)
    x = dev(np.ones(A.n, complex))
    with pytest.raises(hz.HelmzError):
        hz.csr_zspmv(rp, ci, v, x, y=x)


# ---------------------------------------------------------------- BLAS-1


def test_blas1_small_integers_exact(hz):
    x = np.array([1 + 2j, 3 - 1j])
    y = np.array([2 - 1j, 1 + 4j])
    assert complex(hz.zdotc(dev(x), dev(y)).cpu()) == -1 + 8j
    assert complex(hz.zdotc(dev(y), dev(x)).cpu()) == -1 - 8j
    assert float(hz.dznrm2(dev(np.array([3 + 4j, 0j]))).cpu()) == 5.0
    yy = dev(np.array([4 + 0j, 2j]))
    hz.zaxpy(2 - 1j, dev(np.array([1 + 1j, -3 + 0j])), yy)
    assert np.array_equal(yy.cpu().numpy(), np.array([7 + 1j, -6 + 5j]))


@pytest.mark.parametrize("n", [1, 5, 1000, 12345, 209777, 1_500_001])
def test_zdotc_dznrm2_parity(hz, n):
    rng = np.random.default_rng(n)
    x, y = cn(rng, n), cn(rng, n)
    d = complex(hz.zdotc(dev(x), dev(y)).cpu())
    do = O.zdotc(x, y)
    scale = np.sum(np.abs(x) * np.abs(y))
    assert abs(d - do) <= max(n, 16) * EPS * scale
    nr = float(hz.dznrm2(dev(x)).cpu())
    assert abs(nr - O.dznrm2(x)) <= max(n, 16) * EPS * O.dznrm2(x)
    # deterministic
    assert complex(hz.zdotc(dev(x), dev(y)).cpu()) == d


@pytest.mark.parametrize("n", [1, 3, 12345, 209777])
def test_zaxpy_parity(hz, n):
    rng = np.random.default_rng(n + 7)
    x, y = cn(rng, n), cn(rng, n)
    alpha = 0.7 - 0.3j
    out = hz.zaxpy(alpha, dev(x), dev(y)).cpu().numpy()
    ref = O.zaxpy(alpha, x, y)
    bound = 4 * EPS * (np.abs(alpha) * np.abs(x) + np.abs(y))
    assert np.all(np.abs(out - ref) <= bound)


# ---------------------------------------------------------------- BiCGStab


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


def test_solve_cube_matches_oracle(hz):
    A, b, _ = W.config_cube(20)
    tol = 1e-8
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=tol, maxiter=20000)
    x = x.cpu().numpy()
    xo, io = O.zbicgstab(A, b, tol=tol)
    assert info["status"] == hz.OK and io["status"] == O.OK
    rr = true_relres(A, x, b)
    assert rr <= tol * (1 + 1e-3), rr
    assert abs(info["relres_true"] - rr) <= 1e-3 * rr
    assert abs(info["iterations"] - io["iterations"]) <= max(3, 0.1 * io["iterations"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-4


@pytest.mark.parametrize("jacobi", [False, True])
def test_solve_small_systems_match_dense_lu(hz, jacobi):
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    for A, b in [W.config_cube(10, seed=3)[:2], W.config_cylinder(h=1 / 3, k=3.0, seed=1)[:2]]:
        rp, ci, v = dev_csr(A)
        tol = 1e-10
        x, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=tol, flags=flags)
        assert info["status"] == hz.OK
        x = x.cpu().numpy()
        D = O.to_dense(A)
        assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= tol * (1 + 1e-3)
        xd = np.linalg.solve(D, b)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * np.linalg.cond(D) * tol


def test_solve_is_deterministic(hz):
    A, b, _ = W.config_cube(12, seed=9)
    rp, ci, v = dev_csr(A)
    x1, i1 = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-9, flags=hz.PRECOND_JACOBI)
    x2, i2 = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-9, flags=hz.PRECOND_JACOBI)
    assert i1 == i2
    assert torch.equal(torch.view_as_real(x1), torch.view_as_real(x2))


def test_solve_special_cases(hz):
    A, b, _ = W.config_cube(6)
    rp, ci, v = dev_csr(A)
    # b = 0 -> x = 0 regardless of the initial guess
    x0 = dev(np.ones(A.n, complex))
    x, info = hz.zbicgstab_solve(rp, ci, v, dev(np.zeros(A.n, complex)), x=x0, flags=hz.PRECOND_NONE)
    assert info["status"] == hz.OK and info["iterations"] == 0 and torch.count_nonzero(x) == 0
    # maxiter = 1
    _, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-14, maxiter=1)
    assert info["status"] == hz.NOT_CONVERGED and info["iterations"] == 1
    # NaN in b
    bn = b.copy()
    bn[4] = np.nan
    _, info = hz.zbicgstab_solve(rp, ci, v, dev(bn), rtol=1e-8)
    assert info["status"] == hz.NONFINITE
    # warm start at the solution: converged before the first iteration
    xs = np.linalg.solve(O.to_dense(A), b)
    x, info = hz.zbicgstab_solve(rp, ci, v, dev(b), x=dev(xs), rtol=1e-8, flags=hz.PRECOND_NONE)
    assert info["status"] == hz.OK and info["iterations"] == 0


def test_solve_breakdown_and_invalid(hz):
    Z = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
    rp, ci, v = dev_csr(Z)
    _, info = hz.zbicgstab_solve(rp, ci, v, dev(np.array([1.0 + 0j, 0j])), rtol=1e-8)
    assert info["status"] == hz.BREAKDOWN and info["iterations"] == 1 and info["breakdown"] == hz.BD_RHAT_V
    with pytest.raises(hz.HelmzError) as e:
        hz.zbicgstab_solve(rp, ci, v, dev(np.ones(2, complex)), rtol=1e-8, flags=hz.PRECOND_JACOBI)
    assert e.value.code == -1
    # malformed CSR (column out of range) is rejected by device validation before any product
    bad = CSR(np.array([0, 1, 2], np.int32), np.array([0, 5], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
    rp, ci, v = dev_csr(bad)
    with pytest.raises(hz.HelmzError) as e:
        hz.zbicgstab_solve(rp, ci, v, dev(np.ones(2, complex)), flags=hz.VALIDATE)
    assert e.value.code == -1


def test_solve_cylinder_full_size_jacobi(hz):
    A, b, _ = W.config_cylinder()
    tol = 1e-8
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=tol, maxiter=20000, flags=hz.PRECOND_JACOBI)
    assert info["status"] == hz.OK, info
    rr = true_relres(A, x.cpu().numpy(), b)
    print(f"cylinder n={A.n} nnz={A.nnz} iterations={info['iterations']} true relres={rr:.3e}")
    assert rr <= tol * (1 + 1e-3)


@pytest.mark.parametrize("jacobi", [False, True])
def test_solve_both_iteration_variants(hz, jacobi, monkeypatch):
    """The fused (3-kernel) and gather-light (5-kernel) iterations compute the same iterates.

    Iteration counts of BiCGStab on these indefinite systems are chaotic under
    rounding (the oracle itself moves from 668 to 502 iterations on the small
    cylinder below when b or A is perturbed by 1e-16 relative), so the GPU is
    not held to the oracle's count.  The two GPU variants form identical
    vectors (only the summation order of ||s||^2 differs), so they must agree
    with each other to within one iteration, and both must meet the tolerance.
    """
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    for A, b in [W.config_cube(12, seed=4)[:2], W.config_cylinder(h=0.1, k=8.0, seed=2)[:2]]:
        rp, ci, v = dev_csr(A)
        out = {}
        for fused in ("1", "0"):
            monkeypatch.setenv("HZ_FUSED", fused)
            x, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-9, flags=flags)
            assert info["status"] == hz.OK, info
            x = x.cpu().numpy()
            assert true_relres(A, x, b) <= 1e-9 * (1 + 1e-3)
            out[fused] = (x, info["iterations"])
        assert abs(out["1"][1] - out["0"][1]) <= 1, (out["1"][1], out["0"][1])
        assert np.linalg.norm(out["1"][0] - out["0"][0]) / np.linalg.norm(out["0"][0]) <= 1e-6
    for fused in ("1", "0"):
        monkeypatch.setenv("HZ_FUSED", fused)
        Z = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
        rp, ci, v = dev_csr(Z)
        _, info = hz.zbicgstab_solve(rp, ci, v, dev(np.array([1.0 + 0j, 0j])), rtol=1e-8)
        assert info["status"] == hz.BREAKDOWN and info["iterations"] == 1 and info["breakdown"] == hz.BD_RHAT_V
        A, b, _ = W.config_cube(6)
        rp, ci, v = dev_csr(A)
        _, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-14, maxiter=3)
        assert info["status"] == hz.NOT_CONVERGED and info["iterations"] == 3


def test_solve_cabin_full_size_permuted(hz):
    """Randomly numbered cabin (1.24M rows): Jacobi-BiCGStab to 1e-8, checked with the oracle SpMV."""
    A, b, info = W.config_cabin()
    rp, ci, v = dev_csr(A)
    x, sinfo = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-8, maxiter=50000, flags=hz.PRECOND_JACOBI)
    assert sinfo["status"] == hz.OK, sinfo
    assert sinfo["renumbered"] == 1  # the random numbering is replaced by level sets
    x = x.cpu().numpy()
    rr = true_relres(A, x, b)
    print(f"cabin n={A.n} nnz={A.nnz} iterations={sinfo['iterations']} true relres={rr:.3e}")
    assert rr <= 1e-8 * (1 + 1e-3)
    # un-permuted, the solution satisfies the original system too
    A0, b0, _ = W.config_cabin(permute=False)
    x0 = np.empty_like(x)
    x0[:] = x[info["perm"]]
    assert true_relres(A0, x0, b0) <= 1e-8 * (1 + 1e-3)
