"""GPU parity of shared-pattern batched solves (a frequency sweep on one mesh).

Each member must meet its tolerance on its own system (true residual by the
oracle's SpMV) and agree with the single-system solve of the same system;
a member's arithmetic does not depend on the others, so permuting the batch
permutes the results bitwise.  Every lane width (B <= 16, <= 64, <= 256)
and a ragged number of rows are exercised.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from workloads.csr import CSR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def solve_multi(hz, A, vals, rhs, tol, flags, maxiter=20000, x0=None):
    """vals (B, nnz), rhs (B, n) -> list of x_j, infos."""
    V = dev(np.ascontiguousarray(vals.T))
    Bm = dev(np.ascontiguousarray(rhs.T))
    x = None if x0 is None else dev(np.ascontiguousarray(x0.T))
    xs, infos = hz.zbicgstab_solve_batched(dev(A.row_ptr), dev(A.col_idx), V, Bm, x=x, rtol=tol, maxiter=maxiter,
                                           flags=flags)
    xs = xs.cpu().numpy()
    return [xs[:, j].copy() for j in range(vals.shape[0])], infos


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


def sweep(B, h=0.1, kmin=4.0, kmax=9.0, seed=0):
    A, vals, rhs, ks, _ = W.config_freq_sweep(B=B, h=h, kmin=kmin, kmax=kmax, seed=seed)
    return A, vals, rhs


def test_each_member_meets_tolerance_and_matches_single_solve(hz):
    A, vals, rhs = sweep(6)
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-9, hz.PRECOND_JACOBI)
    for j in range(6):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK, infos[j]
        assert true_relres(Aj, xs[j], rhs[j]) <= 1e-9 * (1 + 1e-3)
        x1, i1 = hz.zbicgstab_solve(dev(A.row_ptr), dev(A.col_idx), dev(vals[j]), dev(rhs[j]), rtol=1e-9,
                                    flags=hz.PRECOND_JACOBI)
        x1 = x1.cpu().numpy()
        assert np.linalg.norm(xs[j] - x1) / np.linalg.norm(x1) < 1e-6
        # iteration counts are not compared: on these indefinite systems they move by up to a quarter under
        # perturbations at the rounding level (the oracle's own count does), so only x and residuals are unique
        print(f"k-system {j}: batched {infos[j]['iterations']} iterations, single {i1['iterations']}")
        assert abs(infos[j]["relres_true"] - true_relres(Aj, xs[j], rhs[j])) <= 1e-3 * infos[j]["relres_true"] + 1e-15


def test_members_match_the_oracle_solver(hz):
    A, vals, rhs = sweep(3, h=0.15, seed=2)
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-10, hz.PRECOND_JACOBI)
    for j in range(3):
        Aj = A.with_vals(vals[j])
        xo, io = O.zbicgstab(Aj, rhs[j], tol=1e-10, jacobi=True)
        assert io["status"] == O.OK and infos[j]["status"] == hz.OK
        xd = np.linalg.solve(O.to_dense(Aj), rhs[j])
        kappa = np.linalg.cond(O.to_dense(Aj))
        for x in (xs[j], xo):
            assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * kappa * 1e-10


@pytest.mark.parametrize("B", [1, 5, 17, 64, 65, 256])
def test_every_lane_width_and_ragged_rows(hz, B):
    """Cube N=7 (343 rows: not a multiple of any rows-per-step), B systems with their own k."""
    A0 = W.helmholtz_cube(7)
    rng = np.random.default_rng(B)
    ks = rng.uniform(8.0, 14.0, size=B)
    vals = np.empty((B, A0.nnz), complex)
    rhs = np.empty((B, A0.n), complex)
    for j, k in enumerate(ks):
        vals[j] = W.helmholtz_cube(7, k=k).vals
        rhs[j] = rng.standard_normal(A0.n) + 1j * rng.standard_normal(A0.n)
    xs, infos = solve_multi(hz, A0, vals, rhs, 1e-10, hz.PRECOND_NONE)
    for j in range(B):
        assert infos[j]["status"] == hz.OK, (j, infos[j])
        assert true_relres(A0.with_vals(vals[j]), xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)


def test_permuting_the_batch_permutes_results_bitwise(hz):
    A, vals, rhs = sweep(5, seed=4)
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-9, hz.PRECOND_JACOBI)
    order = [3, 0, 4, 1, 2]
    xp, ip = solve_multi(hz, A, vals[order], rhs[order], 1e-9, hz.PRECOND_JACOBI)
    for pos, k in enumerate(order):
        assert ip[pos] == infos[k]
        assert np.array_equal(xp[pos].view(np.float64), xs[k].view(np.float64))
    # and a rerun is bitwise identical
    xr, ir = solve_multi(hz, A, vals, rhs, 1e-9, hz.PRECOND_JACOBI)
    assert ir == infos and all(np.array_equal(a.view(np.float64), b.view(np.float64)) for a, b in zip(xr, xs))


def test_each_system_reports_its_own_status(hz):
    """Breakdown, zero right-hand side and convergence side by side; then the iteration limit."""
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    P = CSR(rp, ci, np.zeros(4, complex))
    vals = np.array([[0, 1, 1, 0], [2, 1, 1, 3], [2, 1, 1, 3]], complex)  # [[0,1],[1,0]] breaks down on e1
    rhs = np.array([[1, 0], [1, 1], [0, 0]], complex)
    xs, infos = solve_multi(hz, P, vals, rhs, 1e-12, hz.PRECOND_NONE)
    assert infos[0]["status"] == hz.BREAKDOWN and infos[0]["iterations"] == 1
    assert infos[0]["breakdown"] == hz.BD_RHAT_V and infos[1]["breakdown"] == hz.BD_NONE
    assert infos[1]["status"] == hz.OK
    assert np.allclose(xs[1], np.linalg.solve(vals[1].reshape(2, 2), rhs[1]), rtol=1e-12)
    assert infos[2]["status"] == hz.OK and infos[2]["iterations"] == 0 and np.all(xs[2] == 0)
    A, v, r = sweep(2, seed=1)
    _, infos = solve_multi(hz, A, v, r, 1e-14, hz.PRECOND_JACOBI, maxiter=5)
    assert [i["status"] for i in infos] == [hz.NOT_CONVERGED] * 2 and [i["iterations"] for i in infos] == [5, 5]


def test_initial_guess_is_used(hz):
    A, vals, rhs = sweep(4, seed=3)
    xa, _ = solve_multi(hz, A, vals, rhs, 1e-4, hz.PRECOND_JACOBI)
    x0 = np.stack(xa)
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-10, hz.PRECOND_JACOBI, x0=x0)
    _, cold = solve_multi(hz, A, vals, rhs, 1e-10, hz.PRECOND_JACOBI)
    for j in range(4):
        assert infos[j]["status"] == hz.OK
        assert infos[j]["iterations"] < cold[j]["iterations"]
        assert true_relres(A.with_vals(vals[j]), xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)


def test_zero_diagonal_with_jacobi_is_invalid(hz):
    A, vals, rhs = sweep(3, seed=5)
    vals = vals.copy()
    d = np.flatnonzero(A.col_idx == A.row_of_entry())[7]
    vals[1, d] = 0.0
    with pytest.raises(hz.HelmzError) as e:
        solve_multi(hz, A, vals, rhs, 1e-8, hz.PRECOND_JACOBI)
    assert e.value.code == -1


def test_full_size_cylinder_frequency_sweep(hz):
    """64 wavenumbers k ~ U[10, 40] on the cylinder pattern (n=209,777): Jacobi-BiCGStab to 1e-8 each."""
    A, vals, rhs, ks, _ = W.config_freq_sweep(B=64)
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-8, hz.PRECOND_JACOBI, maxiter=50000)
    its = []
    for j in range(64):
        assert infos[j]["status"] == hz.OK, (j, ks[j], infos[j])
        assert true_relres(A.with_vals(vals[j]), xs[j], rhs[j]) <= 1e-8 * (1 + 1e-3)
        its.append(infos[j]["iterations"])
    print(f"frequency sweep B=64 n={A.n}: iterations min {min(its)} max {max(its)}")


def solve_sweep(hz, A, info, ks, rhs, tol, flags, maxiter=20000, x0=None):
    K, M, Bm = (dev(info[k]) for k in ("K", "M", "B"))
    x = None if x0 is None else dev(np.ascontiguousarray(x0.T))
    xs, infos = hz.zbicgstab_solve_sweep(dev(A.row_ptr), dev(A.col_idx), K, M, Bm, ks, dev(np.ascontiguousarray(rhs.T)),
                                         x=x, rtol=tol, maxiter=maxiter, flags=flags)
    xs = xs.cpu().numpy()
    return [xs[:, j].copy() for j in range(len(ks))], infos


@pytest.mark.parametrize("jacobi", [False, True])
def test_sweep_from_three_matrices_matches_explicit_values(hz, jacobi):
    """K - k^2 M + i k B formed in the kernels: same solutions as the batch with explicit values."""
    A, vals, rhs, ks, info = W.config_freq_sweep(B=6, h=0.1, kmin=4.0, kmax=9.0, seed=6)
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    xs, infos = solve_sweep(hz, A, info, ks, rhs, 1e-10, flags)
    xe, ie = solve_multi(hz, A, vals, rhs, 1e-10, flags)
    for j in range(6):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK, infos[j]
        assert true_relres(Aj, xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
        assert np.linalg.norm(xs[j] - xe[j]) / np.linalg.norm(xe[j]) < 1e-7
        assert abs(infos[j]["relres_true"] - true_relres(Aj, xs[j], rhs[j])) <= 1e-3 * infos[j]["relres_true"] + 1e-16


def test_sweep_initial_guess_and_invalid_wavenumber(hz):
    A, vals, rhs, ks, info = W.config_freq_sweep(B=3, h=0.15, kmin=3.0, kmax=6.0, seed=7)
    xa, _ = solve_sweep(hz, A, info, ks, rhs, 1e-4, hz.PRECOND_JACOBI)
    xs, infos = solve_sweep(hz, A, info, ks, rhs, 1e-10, hz.PRECOND_JACOBI, x0=np.stack(xa))
    _, cold = solve_sweep(hz, A, info, ks, rhs, 1e-10, hz.PRECOND_JACOBI)
    for j in range(3):
        assert infos[j]["status"] == hz.OK and infos[j]["iterations"] < cold[j]["iterations"]
        assert true_relres(A.with_vals(vals[j]), xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
    bad = np.array(ks, dtype=float)
    bad[1] = np.nan
    with pytest.raises(hz.HelmzError) as e:
        solve_sweep(hz, A, info, bad, rhs, 1e-8, hz.PRECOND_JACOBI)
    assert e.value.code == -1


def test_sweep_of_more_than_16_systems_runs_in_groups(hz):
    """More than 16 wavenumbers run as groups of neighbouring wavenumbers, one group after another: every member
    meets the tolerance (oracle product), agrees with the explicit-value batch, uses its initial guess, and
    permuting the systems permutes the results bitwise (the groups follow the sorted wavenumbers)."""
    B = 20
    A, vals, rhs, ks, info = W.config_freq_sweep(B=B, h=0.12, kmin=3.0, kmax=9.0, seed=8)
    flags = hz.PRECOND_JACOBI
    xs, infos = solve_sweep(hz, A, info, ks, rhs, 1e-10, flags)
    xe, _ = solve_multi(hz, A, vals, rhs, 1e-10, flags)
    for j in range(B):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK, infos[j]
        assert true_relres(Aj, xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
        assert np.linalg.norm(xs[j] - xe[j]) / np.linalg.norm(xe[j]) < 1e-7
    perm = np.random.default_rng(3).permutation(B)
    xp, ip = solve_sweep(hz, A, info, ks[perm], rhs[perm], 1e-10, flags)
    for k, j in enumerate(perm):
        assert np.array_equal(xp[k].view(np.float64), xs[j].view(np.float64))
        assert ip[k]["iterations"] == infos[j]["iterations"]
    # a warm start from a loose solve takes fewer iterations in every group
    xa, _ = solve_sweep(hz, A, info, ks, rhs, 1e-4, flags)
    xw, iw = solve_sweep(hz, A, info, ks, rhs, 1e-10, flags, x0=np.stack(xa))
    for j in range(B):
        assert iw[j]["status"] == hz.OK and iw[j]["iterations"] < infos[j]["iterations"]
        assert true_relres(A.with_vals(vals[j]), xw[j], rhs[j]) <= 1e-10 * (1 + 1e-3)


def test_full_size_cylinder_sweep_from_three_matrices(hz):
    """64 wavenumbers k ~ U[10, 40] on the cylinder (n=209,777) from K, M, B: Jacobi-BiCGStab to 1e-8 each."""
    A, vals, rhs, ks, info = W.config_freq_sweep(B=64)
    xs, infos = solve_sweep(hz, A, info, ks, rhs, 1e-8, hz.PRECOND_JACOBI, maxiter=50000)
    its = []
    for j in range(64):
        assert infos[j]["status"] == hz.OK, (j, ks[j], infos[j])
        assert true_relres(A.with_vals(vals[j]), xs[j], rhs[j]) <= 1e-8 * (1 + 1e-3)
        its.append(infos[j]["iterations"])
    print(f"K/M/B sweep B=64 n={A.n}: iterations min {min(its)} max {max(its)}")


def long_row_kmb(n=3000, long_rows=(100, 2000), width=1600, seed=9):
    """K, M, B on one pattern with two rows of `width` entries: the 64-row tiles holding them exceed the
    1,536 entries that the K/M/B products stage in LDS, so those tiles take the per-lane path."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    offs = [-7, -1, 1, 7]
    K = sp.diags([np.full(n, 10.0)] + [np.full(n - abs(o), -0.1) for o in offs], [0] + offs, format="lil")
    for r in long_rows:
        for c in rng.choice(n, size=width, replace=False):
            if c != r:
                K[r, c] = K[r, c] + 1e-4
    K = K.tocsr()
    K.sort_indices()
    rows = np.repeat(np.arange(n), np.diff(K.indptr))
    diag = rows == K.indices
    M = np.where(diag, 0.1, 0.0)
    Bv = np.where(diag, 0.05, 0.0)
    A = CSR(K.indptr.astype(np.int32), K.indices.astype(np.int32), K.data.astype(np.complex128))
    return A, {"K": K.data.copy(), "M": M, "B": Bv}


@pytest.mark.parametrize("jacobi", [False, True])
def test_sweep_with_tiles_too_long_to_stage(hz, jacobi):
    A, info = long_row_kmb()
    assert np.diff(A.row_ptr).max() >= 1536
    B = 16
    ks = np.linspace(1.0, 2.0, B)
    vals = np.stack([info["K"] - k * k * info["M"] + 1j * k * info["B"] for k in ks])
    rng = np.random.default_rng(10)
    rhs = rng.standard_normal((B, A.n)) + 1j * rng.standard_normal((B, A.n))
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    xs, infos = solve_sweep(hz, A, info, ks, rhs, 1e-10, flags)
    xe, _ = solve_multi(hz, A, vals, rhs, 1e-10, flags)
    for j in range(B):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK, infos[j]
        assert true_relres(Aj, xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
        assert np.linalg.norm(xs[j] - xe[j]) / np.linalg.norm(xe[j]) < 1e-8


@pytest.mark.parametrize("jacobi", [False, True])
def test_batch_of_more_than_16_systems_runs_in_groups_by_diagonal(hz, jacobi):
    """More than 16 explicit value sets run as groups of up to 16 in order of the mean real diagonal (for a sweep,
    the wavenumbers): every member meets the tolerance (oracle product) and agrees with its single-system solve,
    an initial guess is used, and permuting the systems permutes the results bitwise (the groups follow the keys,
    not the positions)."""
    B = 24
    A, vals, rhs, ks, _ = W.config_freq_sweep(B=B, h=0.12, kmin=3.0, kmax=9.0, seed=11)
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    xs, infos = solve_multi(hz, A, vals, rhs, 1e-10, flags)
    for j in range(B):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK, (j, infos[j])
        assert true_relres(Aj, xs[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
    for j in (0, 7, 23):
        x1, i1 = hz.zbicgstab_solve(dev(A.row_ptr), dev(A.col_idx), dev(vals[j]), dev(rhs[j]), rtol=1e-10,
                                    flags=flags | hz.X0_ZERO)
        x1 = x1.cpu().numpy()
        assert np.linalg.norm(xs[j] - x1) / np.linalg.norm(x1) < 1e-7
    perm = np.random.default_rng(12).permutation(B)
    xp, ip = solve_multi(hz, A, vals[perm], rhs[perm], 1e-10, flags)
    for k, j in enumerate(perm):
        assert np.array_equal(xp[k].view(np.float64), xs[j].view(np.float64))
        assert ip[k] == infos[j]
    xa, _ = solve_multi(hz, A, vals, rhs, 1e-4, flags)
    xw, iw = solve_multi(hz, A, vals, rhs, 1e-10, flags, x0=np.stack(xa))
    for j in range(B):
        assert iw[j]["status"] == hz.OK and iw[j]["iterations"] < infos[j]["iterations"]
        assert true_relres(A.with_vals(vals[j]), xw[j], rhs[j]) <= 1e-10 * (1 + 1e-3)
