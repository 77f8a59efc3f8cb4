"""GPU parity of batched solves (independent systems in one launch sequence).

Each member must meet its tolerance on its own system (true residual by the
oracle's SpMV); a batch of one must equal the single solve bitwise; the
work split of a member does not depend on its neighbours, so permuting the
batch permutes the results bitwise.
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


def block_diag(systems):
    """Concatenate (A_j, b_j) into one block-diagonal CSR with global column indices."""
    row_off = np.zeros(len(systems) + 1, dtype=np.int64)
    rps, cis, vs, bs = [], [], [], []
    nnz_off = 0
    for j, (A, b) in enumerate(systems):
        row_off[j + 1] = row_off[j] + A.n
        rps.append(A.row_ptr[:-1].astype(np.int64) + nnz_off)
        cis.append(A.col_idx.astype(np.int64) + row_off[j])
        vs.append(A.vals)
        bs.append(b)
        nnz_off += A.nnz
    rp = np.concatenate(rps + [np.array([nnz_off])]).astype(np.int32)
    return row_off.astype(np.int32), CSR(rp, np.concatenate(cis).astype(np.int32), np.concatenate(vs)), np.concatenate(bs)


def solve_batch(hz, systems, tol, flags, maxiter=20000):
    row_off, A, b = block_diag(systems)
    x, infos = hz.zbicgstab_solve_varbatch(row_off, dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b), rtol=tol,
                                          maxiter=maxiter, flags=flags)
    x = x.cpu().numpy()
    return [x[row_off[j]:row_off[j + 1]] for j in range(len(systems))], infos


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


def test_batch_of_one_equals_single_solve(hz):
    A, b, _ = W.config_cube(12, seed=3)
    xs, infos = solve_batch(hz, [(A, b)], 1e-9, hz.PRECOND_JACOBI)
    x1, i1 = hz.zbicgstab_solve(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b), rtol=1e-9, flags=hz.PRECOND_JACOBI)
    assert infos[0] == i1
    assert np.array_equal(xs[0].view(np.float64), x1.cpu().numpy().view(np.float64))


@pytest.mark.parametrize("jacobi", [False, True])
def test_uneven_cubes_each_meet_tolerance(hz, jacobi):
    systems, info = W.config_cube_batch(B=7, nmin=4, nmax=11, seed=5)
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    xs, infos = solve_batch(hz, systems, 1e-10, flags)
    for (A, b), x, inf in zip(systems, xs, infos):
        assert inf["status"] == hz.OK, inf
        assert true_relres(A, x, b) <= 1e-10 * (1 + 1e-3)
        xd = np.linalg.solve(O.to_dense(A), b)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * np.linalg.cond(O.to_dense(A)) * 1e-10
    # different sizes converge after different numbers of iterations
    assert len({inf["iterations"] for inf in infos}) > 1


def test_batch_permutation_permutes_results_bitwise(hz):
    systems, _ = W.config_cube_batch(B=5, nmin=6, nmax=12, seed=8)
    xs, infos = solve_batch(hz, systems, 1e-9, hz.PRECOND_JACOBI)
    order = [3, 0, 4, 1, 2]
    xp, ip = solve_batch(hz, [systems[k] for k in order], 1e-9, hz.PRECOND_JACOBI)
    for pos, k in enumerate(order):
        assert ip[pos] == infos[k]
        assert np.array_equal(xp[pos].view(np.float64), xs[k].view(np.float64))


def test_frequency_sweep_shared_pattern(hz):
    A, vals, rhs, ks, _ = W.config_freq_sweep(B=6, h=0.1, kmin=4.0, kmax=9.0)
    systems = [(A.with_vals(vals[j]), rhs[j]) for j in range(len(ks))]
    xs, infos = solve_batch(hz, systems, 1e-9, hz.PRECOND_JACOBI)
    for (Aj, bj), x, inf in zip(systems, xs, infos):
        assert inf["status"] == hz.OK, inf
        assert true_relres(Aj, x, bj) <= 1e-9 * (1 + 1e-3)


def test_batch_reports_each_status(hz):
    """A breakdown or an iteration limit in one member does not stop the others."""
    Z = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0 + 0j, 1.0 + 0j]))
    A, b, _ = W.config_cube(6, seed=2)
    A2, b2, _ = W.config_cube(9, seed=4)
    systems = [(A, b), (Z, np.array([1.0 + 0j, 0j])), (A2, b2), (A, np.zeros(A.n, complex))]
    xs, infos = solve_batch(hz, systems, 1e-9, hz.PRECOND_NONE)
    assert infos[0]["status"] == hz.OK and true_relres(A, xs[0], b) <= 1e-9 * (1 + 1e-3)
    assert infos[1]["status"] == hz.BREAKDOWN and infos[1]["iterations"] == 1
    assert infos[1]["breakdown"] == hz.BD_RHAT_V and infos[0]["breakdown"] == hz.BD_NONE
    assert infos[2]["status"] == hz.OK and true_relres(A2, xs[2], b2) <= 1e-9 * (1 + 1e-3)
    assert infos[3]["status"] == hz.OK and infos[3]["iterations"] == 0 and np.all(xs[3] == 0)
    _, infos = solve_batch(hz, systems[:1] + systems[2:3], 1e-12, hz.PRECOND_NONE, maxiter=5)
    assert [i["status"] for i in infos] == [hz.NOT_CONVERGED] * 2
    assert [i["iterations"] for i in infos] == [5, 5]


def test_full_uneven_cube_batch(hz):
    """32 cubes with N ~ U{16..64}, each with its own k, unpreconditioned BiCGStab to 1e-8."""
    systems, info = W.config_cube_batch(B=32)
    xs, infos = solve_batch(hz, systems, 1e-8, hz.PRECOND_NONE, maxiter=50000)
    its = []
    for (A, b), x, inf in zip(systems, xs, infos):
        assert inf["status"] == hz.OK, inf
        assert true_relres(A, x, b) <= 1e-8 * (1 + 1e-3)
        its.append(inf["iterations"])
    print(f"cube batch: sum n = {sum(A.n for A, _ in systems)}, iterations min {min(its)} max {max(its)}")
