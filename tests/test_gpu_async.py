"""The asynchronous solve (zbicgstab_solve_async) against the synchronous one.

Both run the same kernels on the same map; the asynchronous call enqueues
every chunk without polling (kernels after the exit return at entry) and
writes hz_solve_info from the device, so x must be bitwise equal and the
info identical.  Two solves enqueued back to back before any host wait must
both be right; the oracle's true residual checks the solutions.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("jacobi", [False, True])
def test_async_equals_sync(hz, jacobi):
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = (hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE) | hz.X0_ZERO | hz.NO_REORDER
    xs, is_ = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, maxiter=3000, flags=flags)
    xa, info = hz.zbicgstab_solve_async(rp, ci, v, bd, rtol=1e-10, maxiter=3000, flags=flags & ~hz.NO_REORDER)
    ia = hz.read_info(info)
    assert ia == is_, (ia, is_)
    assert np.array_equal(xa.cpu().numpy().view(np.float64), xs.cpu().numpy().view(np.float64))
    assert ia["status"] == hz.OK and true_relres(A, xa.cpu().numpy(), b) <= 1e-10 * (1 + 1e-2)


def test_two_solves_enqueued_before_any_wait(hz):
    A, b, _ = W.config_cube(12, seed=2)
    rng = np.random.default_rng(4)
    b2 = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    x1, i1 = hz.zbicgstab_solve_async(rp, ci, v, dev(b), rtol=1e-10, maxiter=2000)
    x2, i2 = hz.zbicgstab_solve_async(rp, ci, v, dev(b2), rtol=1e-10, maxiter=2000)
    torch.cuda.synchronize()
    for x, info, rhs in ((x1, i1, b), (x2, i2, b2)):
        d = hz.read_info(info)
        assert d["status"] == hz.OK and d["renumbered"] == 0
        assert true_relres(A, x.cpu().numpy(), rhs) <= 1e-10 * (1 + 1e-2)


def test_iteration_limit_zero_diagonal_and_invalid(hz):
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO | hz.NO_REORDER
    xs, is_ = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-30, maxiter=37, flags=flags)
    xa, info = hz.zbicgstab_solve_async(rp, ci, v, bd, rtol=1e-30, maxiter=37, flags=flags & ~hz.NO_REORDER)
    ia = hz.read_info(info)
    assert ia == is_ and ia["status"] == hz.NOT_CONVERGED and ia["iterations"] == 37
    assert np.array_equal(xa.cpu().numpy().view(np.float64), xs.cpu().numpy().view(np.float64))
    # a zero diagonal entry under Jacobi: reported in the device info
    rows = A.row_of_entry()
    vals = A.vals.copy()
    vals[(A.col_idx == rows) & (rows == 5)] = 0
    _, info = hz.zbicgstab_solve_async(rp, ci, dev(vals), bd, rtol=1e-10, maxiter=50, flags=hz.PRECOND_JACOBI)
    assert hz.read_info(info)["status"] == -1
    for bad in (hz.REORDER, hz.VALIDATE, hz.RELIABLE):
        with pytest.raises(hz.HelmzError):
            hz.zbicgstab_solve_async(rp, ci, v, bd, flags=bad)


def test_many_queued_solves_evict_graphs_safely(hz):
    """20 solves on distinct buffers enqueued before any host wait: about 40 chunk graphs for a cache of 32, so
    graphs are evicted while earlier chunks may still be queued.  Every solution must equal the synchronous
    solve of the same system bit for bit."""
    A, _, _ = W.config_cube(10, seed=3)
    rng = np.random.default_rng(9)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    rhs = [rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n) for _ in range(20)]
    bs = [dev(r) for r in rhs]  # kept alive: distinct buffers give distinct graph keys
    queued = [hz.zbicgstab_solve_async(rp, ci, v, bd, rtol=1e-10, maxiter=400) for bd in bs]
    torch.cuda.synchronize()
    for r, (xa, info) in zip(rhs, queued):
        xs, is_ = hz.zbicgstab_solve(rp, ci, v, dev(r), rtol=1e-10, maxiter=400, flags=hz.X0_ZERO | hz.NO_REORDER)
        ia = hz.read_info(info)
        assert ia == is_, (ia, is_)
        assert np.array_equal(xa.cpu().numpy().view(np.float64), xs.cpu().numpy().view(np.float64))
        assert ia["status"] == hz.OK and true_relres(A, xa.cpu().numpy(), r) <= 1e-10 * (1 + 1e-2)
