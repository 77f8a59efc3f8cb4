"""GPU parity of TFQMR (ztfqmr_solve) against the oracle and dense LU.

The GPU runs the same half steps as the oracle with reductions in another
order, so iterates agree to rounding amplified by the Krylov recurrences:
close for a few iterations, then converged solutions are compared by their
true residuals (recomputed with the oracle's SpMV) and against LU.  The
quasi-residual bound is tested after every half step on both sides, so the
iteration counts differ by at most a few.
"""

import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle.tfqmr import tfqmr
from workloads.csr import CSR, csr_from_coo, permute_symmetric

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def solve(hz, A, b, **kw):
    x, info = hz.ztfqmr_solve(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b), **kw)
    return x.cpu().numpy(), info


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ragged_dominant(n=2000, seed=5, maxlen=90):
    """Row lengths 1..maxlen (one row of 400), diagonally dominant: exercises the wide-lane kernels."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen, n)
    lens[7] = 400
    rows, cols, vals = [], [], []
    for i, L in enumerate(lens):
        c = rng.choice(n, size=L, replace=False)
        c = c[c != i]
        rows += [np.full(c.size, i), [i]]
        cols += [c, [i]]
        off = cn(rng, c.size) / (1 + c.size)
        vals += [off, [3.0 + 1.0j]]
    return csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def test_small_cube_matches_dense_lu(hz):
    A, b, _ = W.config_cube(10, seed=1)
    x, info = solve(hz, A, b, rtol=1e-10)
    assert info["status"] == hz.OK, info
    assert true_relres(A, x, b) <= 1e-10 * (1 + 1e-3)
    assert info["relres_true"] <= info["relres_recursive"] * (1 + 1e-6)
    xd = np.linalg.solve(O.to_dense(A), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    xo, io = tfqmr(A, b, tol=1e-10)
    print(f"cube10: iterations gpu {info['iterations']} oracle {io['iterations']}")
    assert abs(info["iterations"] - io["iterations"]) <= max(2, io["iterations"] // 10)


@pytest.mark.parametrize("iters,bound", [(3, 1e-12), (10, 1e-9)])
@pytest.mark.parametrize("jacobi", [False, True])
def test_iterates_follow_the_oracle(hz, iters, bound, jacobi):
    A, b, _ = W.config_cylinder(h=0.1)
    flags = (hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE) | hz.X0_ZERO | hz.NO_REORDER
    x, info = solve(hz, A, b, rtol=1e-30, maxiter=iters, flags=flags)
    xo, io = tfqmr(A, b, tol=1e-30, maxiter=iters, jacobi=jacobi)
    assert info["status"] == hz.NOT_CONVERGED and info["iterations"] == iters == io["iterations"]
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"jacobi={jacobi} after {iters} iterations: rel diff {err:.2e}")
    assert err <= bound
    assert abs(info["relres_recursive"] - io["relres_recursive"]) <= 1e-8 * io["relres_recursive"]


def test_ragged_rows_follow_the_oracle(hz):
    A = ragged_dominant()
    b = cn(np.random.default_rng(2), A.n)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO | hz.NO_REORDER
    x, info = solve(hz, A, b, rtol=1e-30, maxiter=6, flags=flags)
    xo, io = tfqmr(A, b, tol=1e-30, maxiter=6, jacobi=True)
    assert info["iterations"] == 6 == io["iterations"]
    assert np.linalg.norm(x - xo) <= 1e-11 * np.linalg.norm(xo)
    x, info = solve(hz, A, b, rtol=1e-12, flags=flags)
    assert info["status"] == hz.OK and true_relres(A, x, b) <= 1e-12 * (1 + 1e-2)


def test_half_step_exit_on_a_scaled_identity(hz):
    """A = s I converges at the first half step (w_1 = 0): x = b / s in one iteration."""
    n, s = 777, 2.0 - 0.5j
    A = CSR(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, s, complex))
    b = cn(np.random.default_rng(1), n)
    x, info = solve(hz, A, b, rtol=1e-14)
    assert info["status"] == hz.OK and info["iterations"] == 1
    assert np.linalg.norm(x - b / s) <= 1e-14 * np.linalg.norm(b / s)


def test_jacobi_cylinder_converges_like_the_oracle(hz):
    A, b, _ = W.config_cylinder(h=0.08)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    x, info = solve(hz, A, b, rtol=1e-10, flags=flags)
    xo, io = tfqmr(A, b, tol=1e-10, jacobi=True)
    assert info["status"] == hz.OK and io["status"] == O.OK
    assert true_relres(A, x, b) <= 1e-10 * (1 + 1e-2)
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    print(f"cylinder h=0.08: iterations gpu {info['iterations']} oracle {io['iterations']}")
    # the count near the threshold moves with rounding (the oracle alone gives 424 or 434 with
    # different BLAS summation orders): within 10 %, as for every solver here
    assert abs(info["iterations"] - io["iterations"]) <= max(3, io["iterations"] // 10)


def test_full_size_cylinder(hz):
    A, b, _ = W.config_cylinder()
    assert A.n == 209777
    x, info = solve(hz, A, b, rtol=1e-8, flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
    assert info["status"] == hz.OK, info
    rr = true_relres(A, x, b)
    assert rr <= 1e-8 * (1 + 1e-2)
    print(f"full cylinder: iterations {info['iterations']} true relres {rr:.3e}")


def test_full_size_cylinder_robin_on_the_caps_only(hz):
    """The cylinder with Robin conditions on the end caps only (the lateral wall natural Neumann): a nearly
    undamped waveguide on which Jacobi-BiCGStab stagnates near 4e-4.  TFQMR reaches 1e-8; its stopping
    bound guarantees the true residual, recomputed here with the oracle's product."""
    A, b, _ = W.config_cylinder(robin="caps")
    assert A.n == 209777
    x, info = solve(hz, A, b, rtol=1e-8, maxiter=25000, flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
    assert info["status"] == hz.OK, info
    rr = true_relres(A, x, b)
    assert rr <= 1e-8 * (1 + 1e-2)
    print(f"caps-only cylinder: iterations {info['iterations']} true relres {rr:.3e}")


def test_renumbered_scrambled_mesh(hz):
    A, b, _ = W.config_cube(14, seed=4)
    rng = np.random.default_rng(9)
    perm = rng.permutation(A.n)
    P = permute_symmetric(A, perm)
    bp = np.empty_like(b)
    bp[perm] = b  # row perm[i] of P is row i of A
    x, info = solve(hz, P, bp, rtol=1e-10, flags=hz.REORDER | hz.X0_ZERO)
    assert info["status"] == hz.OK and info["renumbered"] == 1
    assert true_relres(P, x, bp) <= 1e-10 * (1 + 1e-2)


def test_special_cases_and_invalid_arguments(hz):
    A, b, _ = W.config_cube(6, seed=2)
    x, info = solve(hz, A, np.zeros(A.n, complex))
    assert info["status"] == hz.OK and info["iterations"] == 0 and not np.any(x)
    xd = np.linalg.solve(O.to_dense(A), b)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    xg, info = hz.ztfqmr_solve(rp, ci, v, dev(b), x=dev(xd), rtol=1e-8, flags=hz.PRECOND_NONE)
    assert info["status"] == hz.OK and info["iterations"] == 0
    xh, info = hz.ztfqmr_solve(rp, ci, v, dev(b), x=dev(0.5 * xd), rtol=1e-11, flags=hz.PRECOND_JACOBI)
    assert info["status"] == hz.OK and true_relres(A, xh.cpu().numpy(), b) <= 1e-11 * (1 + 1e-2)
    _, info = solve(hz, A, b, maxiter=0)
    assert info["status"] == hz.NOT_CONVERGED and info["iterations"] == 0
    for bad in (dict(flags=hz.RELIABLE), dict(rtol=-1.0), dict(maxiter=-1)):
        with pytest.raises(hz.HelmzError):
            solve(hz, A, b, **bad)


def test_deterministic_and_graph_replays_equal_direct_launches(hz):
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    ws = torch.empty(hz.ztfqmr_workspace_bytes(A.n, A.nnz, flags) + 256, dtype=torch.uint8, device="cuda:0")
    os.environ["HZ_NO_GRAPH"] = "1"
    try:
        xe, ie = hz.ztfqmr_solve(rp, ci, v, bd, rtol=1e-10, flags=flags, ws=ws)
        xe = xe.cpu().numpy()
    finally:
        del os.environ["HZ_NO_GRAPH"]
    for _ in range(3):
        xg, ig = hz.ztfqmr_solve(rp, ci, v, bd, rtol=1e-10, flags=flags, ws=ws)
        assert ig == ie
        assert np.array_equal(xg.cpu().numpy().view(np.float64), xe.view(np.float64))
        torch.cuda.synchronize()


@pytest.mark.parametrize("jacobi", [False, True])
def test_gather_light_equals_fused(hz, jacobi):
    """Above about 1e5 rows the third launch splits in two (one gathered vector): same arithmetic, same bits."""
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = (hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE) | hz.X0_ZERO | hz.NO_REORDER
    out = {}
    for fused in ("1", "0"):
        os.environ["HZ_FUSED"] = fused
        try:
            for maxiter in (7, 5000):
                x, info = hz.ztfqmr_solve(rp, ci, v, bd, rtol=1e-10, maxiter=maxiter, flags=flags)
                out[fused, maxiter] = (x.cpu().numpy(), info)
        finally:
            del os.environ["HZ_FUSED"]
    for maxiter in (7, 5000):
        (x1, i1), (x0, i0) = out["1", maxiter], out["0", maxiter]
        assert i1 == i0
        assert np.array_equal(x1.view(np.float64), x0.view(np.float64))
    assert out["0", 5000][1]["status"] == hz.OK
