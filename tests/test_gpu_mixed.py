"""GPU parity of the mixed-precision solve (complex64 inner BiCGStab, complex128 refinement).

The bar is the FP64 one: the true residual of the returned x, recomputed with
the oracle's complex128 SpMV, meets rtol; the error against the FP64 solution
is reported and bounded by the conditioning.
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


def dev_csr(A):
    return dev(A.row_ptr), dev(A.col_idx), dev(A.vals)


def true_relres(A, x, b):
    return np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("jacobi", [False, True])
def test_mixed_cube_reaches_fp64_tolerance(hz, jacobi):
    A, b, _ = W.config_cube(20)
    tol = 1e-10
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=tol, inner_rtol=1e-4, flags=flags)
    assert info["status"] == hz.OK, info
    assert info["outer_steps"] >= 2
    x = x.cpu().numpy()
    rr = true_relres(A, x, b)
    assert rr <= tol * (1 + 1e-3), rr
    assert abs(info["relres_true"] - rr) <= 1e-3 * rr
    xo, io = O.zbicgstab_mixed(A, b, tol=tol, inner_tol=1e-4, jacobi=jacobi)
    assert io["status"] == O.OK
    x64, _ = O.zbicgstab(A, b, tol=1e-12, jacobi=jacobi)
    err = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    print(f"mixed cube jacobi={jacobi}: outer={info['outer_steps']} inner={info['iterations']} "
          f"(oracle {io['outer_steps']}/{io['iterations']}) relres={rr:.2e} err_vs_fp64={err:.2e}")
    assert err < 1e-6


def test_mixed_small_systems_match_dense_lu(hz):
    for A, b in [W.config_cube(10, seed=3)[:2], W.config_cylinder(h=1 / 3, k=3.0, seed=1)[:2]]:
        rp, ci, v = dev_csr(A)
        x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-11, flags=hz.PRECOND_JACOBI)
        assert info["status"] == hz.OK
        D = O.to_dense(A)
        xd = np.linalg.solve(D, b)
        x = x.cpu().numpy()
        assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-11 * (1 + 1e-3)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * np.linalg.cond(D) * 1e-11


def test_mixed_special_cases(hz):
    A, b, _ = W.config_cube(6)
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(np.zeros(A.n, complex)), x=dev(np.ones(A.n, complex)),
                                       flags=hz.PRECOND_NONE)
    assert info["status"] == hz.OK and torch.count_nonzero(x) == 0
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-12, max_outer=0)
    assert info["status"] == hz.NOT_CONVERGED and info["outer_steps"] == 0
    assert torch.count_nonzero(x) == 0
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-12, max_outer=1)
    assert info["status"] == hz.NOT_CONVERGED and info["outer_steps"] == 1


def test_mixed_cylinder_full_size(hz):
    A, b, _ = W.config_cylinder()
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, inner_rtol=1e-4, flags=hz.PRECOND_JACOBI)
    assert info["status"] == hz.OK, info
    rr = true_relres(A, x.cpu().numpy(), b)
    print(f"mixed cylinder: outer={info['outer_steps']} inner={info['iterations']} relres={rr:.2e}")
    assert rr <= 1e-10 * (1 + 1e-3)


@pytest.mark.parametrize("jacobi", [False, True])
def test_reliable_updates_reach_fp64_tolerance(hz, jacobi):
    """One complex64 BiCGStab with reliable FP64 residual updates: FP64 accuracy, fewer iterations than restarts."""
    A, b, _ = W.config_cube(20)
    flags = hz.PRECOND_JACOBI if jacobi else hz.PRECOND_NONE
    rp, ci, v = dev_csr(A)
    xr, ir = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, flags=flags | hz.RELIABLE)
    xi, ii = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, flags=flags)
    x64, i64 = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-12, flags=flags)
    assert ir["status"] == hz.OK and ir["outer_steps"] >= 2
    xr = xr.cpu().numpy()
    assert true_relres(A, xr, b) <= 1e-10 * (1 + 1e-3)
    assert abs(ir["relres_true"] - true_relres(A, xr, b)) <= 1e-3 * ir["relres_true"]
    x64 = x64.cpu().numpy()
    assert np.linalg.norm(xr - x64) / np.linalg.norm(x64) <= 1e-6
    print(f"cube: reliable {ir['iterations']} its / {ir['outer_steps']} updates, "
          f"restarted {ii['iterations']} its / {ii['outer_steps']} corrections")


def test_reliable_updates_special_cases(hz):
    A, b, _ = W.config_cube(8)
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(np.zeros(A.n, complex)), flags=hz.RELIABLE)
    assert info["status"] == hz.OK and torch.count_nonzero(x) == 0
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-14, maxiter=5, flags=hz.RELIABLE)
    assert info["status"] == hz.NOT_CONVERGED
    with pytest.raises(hz.HelmzError):
        hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), inner_rtol=1.0, flags=hz.RELIABLE)
    # an initial guess is used: its residual is where the updates start from
    xa, _ = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-5, flags=hz.RELIABLE)
    xb, ib = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), x=xa.clone(), rtol=1e-10, flags=hz.RELIABLE)
    _, ic = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, flags=hz.RELIABLE)
    assert ib["status"] == hz.OK and ib["iterations"] < ic["iterations"]
    assert true_relres(A, xb.cpu().numpy(), b) <= 1e-10 * (1 + 1e-3)


def test_reliable_updates_renumbered_cabin(hz):
    A, b, _ = W.config_cabin(h=0.05, k=12.0, seed=5)
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10,
                                       flags=hz.PRECOND_JACOBI | hz.RELIABLE | hz.REORDER)
    assert info["status"] == hz.OK and info["renumbered"] == 1
    assert true_relres(A, x.cpu().numpy(), b) <= 1e-10 * (1 + 1e-3)


def test_reliable_updates_cylinder_full_size(hz):
    A, b, _ = W.config_cylinder()
    rp, ci, v = dev_csr(A)
    x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.RELIABLE)
    assert info["status"] == hz.OK, info
    rr = true_relres(A, x.cpu().numpy(), b)
    print(f"reliable cylinder: updates={info['outer_steps']} iterations={info['iterations']} relres={rr:.2e}")
    assert rr <= 1e-10 * (1 + 1e-3)


@pytest.mark.parametrize("reliable", [False, True])
def test_mixed_full_size_cabin(hz, reliable):
    """The full cabin (1.24 M rows, random numbering, renumbered inside the call) to the FP64 tolerance."""
    A, b, _ = W.config_cabin()
    rp, ci, v = dev_csr(A)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO | (hz.RELIABLE if reliable else 0)
    if reliable:
        x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, maxiter=50000, flags=flags)
    else:
        x, info = hz.zbicgstab_solve_mixed(rp, ci, v, dev(b), rtol=1e-10, inner_rtol=1e-4, maxiter=50000, flags=flags)
    assert info["status"] == hz.OK, info
    assert info["renumbered"] == 1
    rr = true_relres(A, x.cpu().numpy(), b)
    print(f"mixed cabin (reliable={reliable}): outer={info['outer_steps']} inner={info['iterations']} relres={rr:.2e}")
    assert rr <= 1e-10 * (1 + 1e-3)
