"""GPU parity of the level-set renumbering and of solves run in it.

The ordering and P A P^T are index work: bit-exact against the oracle
(oracle/reorder.py) on small and medium patterns, and against levels from
scipy's breadth-first search at the cabin's full size.  Solves in the new
numbering must meet the same true-residual bar as solves in the caller's
numbering and return x in the caller's numbering.
"""

import numpy as np
import pytest
import torch

import oracle as O
import oracle.reorder as R
import workloads as W
from workloads.csr import CSR, csr_from_coo, permute_symmetric

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def path_csr(n):
    i = np.arange(n)
    rows = np.concatenate([i, i[1:], i[:-1]])
    cols = np.concatenate([i, i[:-1], i[1:]])
    return csr_from_coo(n, rows, cols, np.ones(rows.size, np.complex128))


def scrambled_cube(N, seed):
    A, b, _ = W.config_cube(N, seed=seed)
    p = np.random.default_rng(seed + 100).permutation(A.n)
    return permute_symmetric(A, p), b[np.argsort(p)]


def two_components():
    a, b = W.helmholtz_cube(5), W.helmholtz_cube(4)
    rp = np.concatenate([b.row_ptr[:-1], a.row_ptr + b.nnz]).astype(np.int32)
    ci = np.concatenate([b.col_idx, a.col_idx + b.n]).astype(np.int32)
    return CSR(rp, ci, np.concatenate([b.vals, a.vals]))


CASES = {
    "single": lambda: CSR(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0 + 0j])),
    "path700": lambda: path_csr(700),  # 700 levels: many chunks of level steps
    "cube12_scrambled": lambda: scrambled_cube(12, 4)[0],
    "two_components": two_components,
    "cabin_small": lambda: W.config_cabin(h=0.06, k=10.0, seed=2)[0],
}


@pytest.mark.parametrize("case", list(CASES))
def test_level_order_and_permute_bitwise(hz, case):
    A = CASES[case]()
    perm_o, inv_o, level_o = R.level_order(A.row_ptr, A.col_idx)
    perm, inv, level = hz.csr_level_order(dev(A.row_ptr), dev(A.col_idx))
    assert np.array_equal(perm.cpu().numpy(), perm_o)
    assert np.array_equal(inv.cpu().numpy(), inv_o)
    assert np.array_equal(level.cpu().numpy(), level_o)
    rp_o, ci_o, v_o = R.permute(A.row_ptr, A.col_idx, A.vals, perm_o, inv_o)
    rp, ci, v = hz.csr_zpermute(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), perm, inv)
    assert np.array_equal(rp.cpu().numpy(), rp_o)
    assert np.array_equal(ci.cpu().numpy(), ci_o)
    assert np.array_equal(v.cpu().numpy().view(np.float64), v_o.view(np.float64))


def test_permute_rejects_a_non_permutation(hz):
    A = W.helmholtz_cube(4)
    perm = torch.arange(A.n, dtype=torch.int32, device="cuda:0")
    inv = perm.clone()
    perm[3] = 5  # 5 twice, 3 never
    with pytest.raises(hz.HelmzError) as e:
        hz.csr_zpermute(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), perm, inv)
    assert e.value.code == -1
    perm[3] = A.n  # out of range
    with pytest.raises(hz.HelmzError):
        hz.csr_zpermute(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), perm, inv)


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


def test_solve_in_level_order_matches_caller_order(hz):
    A, b, _ = W.config_cabin(h=0.05, k=12.0, seed=3)
    args = (dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b))
    # n < 32768: no entry can lie far from the diagonal, so the default keeps the numbering
    xa, ia = hz.zbicgstab_solve(*args, rtol=1e-9, flags=hz.PRECOND_JACOBI)
    xr, ir = hz.zbicgstab_solve(*args, rtol=1e-9, flags=hz.PRECOND_JACOBI | hz.REORDER)
    xn, inn = hz.zbicgstab_solve(*args, rtol=1e-9, flags=hz.PRECOND_JACOBI | hz.NO_REORDER)
    assert ia["renumbered"] == 0 and ir["renumbered"] == 1 and inn["renumbered"] == 0
    assert np.array_equal(xa.cpu().numpy().view(np.float64), xn.cpu().numpy().view(np.float64))
    for x, inf in ((xr, ir), (xn, inn)):
        assert inf["status"] == hz.OK
        assert true_relres(A, x.cpu().numpy(), b) <= 1e-9 * (1 + 1e-3)
    xr, xn = xr.cpu().numpy(), xn.cpu().numpy()
    assert np.linalg.norm(xr - xn) / np.linalg.norm(xn) < 1e-6
    # iteration counts differ by rounding order only and are not compared (they move by up to a quarter
    # on these indefinite systems under rounding-level perturbations)
    print(f"renumbered {ir['iterations']} iterations, caller order {inn['iterations']}")


def test_reordered_solve_keeps_initial_guess_and_is_deterministic(hz):
    A, b = scrambled_cube(10, 6)
    args = (dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b))
    x0, _ = hz.zbicgstab_solve(*args, rtol=1e-4, flags=hz.REORDER)
    x1, i1 = hz.zbicgstab_solve(*args, x=x0.clone(), rtol=1e-10, flags=hz.REORDER)
    x2, i2 = hz.zbicgstab_solve(*args, x=x0.clone(), rtol=1e-10, flags=hz.REORDER)
    assert i1 == i2 and np.array_equal(x1.cpu().numpy().view(np.float64), x2.cpu().numpy().view(np.float64))
    assert true_relres(A, x1.cpu().numpy(), b) <= 1e-10 * (1 + 1e-3)
    xf, iff = hz.zbicgstab_solve(*args, rtol=1e-10, flags=hz.REORDER)
    assert i1["iterations"] < iff["iterations"]  # the guess was used


def test_both_reorder_flags_is_invalid(hz):
    A, b = scrambled_cube(5, 1)
    with pytest.raises(hz.HelmzError):
        hz.zbicgstab_solve(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b), flags=hz.REORDER | hz.NO_REORDER)


def test_mixed_solve_in_level_order(hz):
    A, b, _ = W.config_cabin(h=0.05, k=12.0, seed=4)
    args = (dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b))
    x, inf = hz.zbicgstab_solve_mixed(*args, rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.REORDER)
    assert inf["status"] == hz.OK and inf["renumbered"] == 1 and inf["outer_steps"] >= 2
    assert true_relres(A, x.cpu().numpy(), b) <= 1e-10 * (1 + 1e-3)


def test_adjoint_in_level_order(hz):
    A, b = scrambled_cube(8, 2)
    g = np.random.default_rng(5).standard_normal((A.n, 2)) @ np.array([1, 1j])
    args = (dev(A.row_ptr), dev(A.col_idx), dev(A.vals))
    x, _ = hz.zbicgstab_solve(*args, dev(b), rtol=1e-12, flags=hz.NO_REORDER)
    lr, vr, ir = hz.zbicgstab_adjoint(*args, x, dev(g), rtol=1e-11, flags=hz.REORDER, want_grad_vals=True)
    ln, vn, inn = hz.zbicgstab_adjoint(*args, x, dev(g), rtol=1e-11, flags=hz.NO_REORDER, want_grad_vals=True)
    assert ir["status"] == hz.OK and inn["status"] == hz.OK
    lam = np.linalg.solve(O.to_dense(A).conj().T, g)
    for l in (lr, ln):
        assert np.linalg.norm(l.cpu().numpy() - lam) / np.linalg.norm(lam) < 1e-8


def test_full_size_cabin_level_order_matches_oracle_with_scipy_bfs(hz):
    """Cabin (n=1.24M, randomly numbered): levels and order equal the oracle's, with scipy's BFS distances."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg

    A, _, _ = W.config_cabin()
    G = sp.csr_matrix((np.ones(A.nnz), A.col_idx, A.row_ptr), shape=(A.n, A.n))

    def scipy_bfs(rp, ci, start):
        d = cg.shortest_path(G, unweighted=True, indices=start)
        return np.where(np.isinf(d), -1, d).astype(np.int64)

    perm_o, inv_o, lev_o = R.level_order(A.row_ptr, A.col_idx, bfs=scipy_bfs)
    perm, inv, level = hz.csr_level_order(dev(A.row_ptr), dev(A.col_idx))
    assert np.array_equal(level.cpu().numpy(), lev_o)
    assert np.array_equal(perm.cpu().numpy(), perm_o)
    assert np.array_equal(inv.cpu().numpy(), inv_o)
    rows = A.row_of_entry()
    band = np.abs(inv_o[rows] - inv_o[A.col_idx]).max()
    print(f"cabin: {lev_o.max() + 1} levels, widest {np.bincount(lev_o).max()}, bandwidth after renumbering {band}")
