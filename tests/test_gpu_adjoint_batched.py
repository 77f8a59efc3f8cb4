"""GPU parity of the batched backward (shared-pattern batches).

References: dense LAPACK solves of A_j^H lambda_j = g_j on small systems, the
oracle's entry-gradient formula per system, and the single-system backward
of the same systems through autograd.
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


def cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def small_sweep(B, nonsym=False, seed=0):
    A, vals, rhs, ks, _ = W.config_freq_sweep(B=B, h=0.2, kmin=3.0, kmax=6.0, seed=seed)
    if nonsym:  # break A = A^T: perturb the strictly upper entries of every system
        upper = A.col_idx > A.row_of_entry()
        vals = vals + 0.05j * upper[None, :] * (1 + np.arange(B) % 5)[:, None]  # the same five sizes for any B
    return A, vals, rhs


@pytest.mark.parametrize("B", [5, 20, 70])  # one launch of 16, 64 and 256 lanes per row
@pytest.mark.parametrize("nonsym", [False, True])
def test_batched_adjoint_matches_dense_and_oracle_gradients(hz, nonsym, B):
    A, vals, rhs = small_sweep(B, nonsym=nonsym, seed=1)
    rng = np.random.default_rng(2)
    G = cn(rng, A.n, B)
    X = np.stack([np.linalg.solve(O.to_dense(A.with_vals(vals[j])), rhs[j]) for j in range(B)], axis=1)
    flags = hz.PRECOND_JACOBI | (0 if nonsym else hz.SYMMETRIC)
    lam, gv, infos = hz.zbicgstab_adjoint_batched(dev(A.row_ptr), dev(A.col_idx), dev(vals.T), dev(X), dev(G),
                                                  rtol=1e-12, flags=flags)
    lam, gv = lam.cpu().numpy(), gv.cpu().numpy()
    for j in range(B):
        Aj = A.with_vals(vals[j])
        assert infos[j]["status"] == hz.OK
        D = O.to_dense(Aj).conj().T
        ld = np.linalg.solve(D, G[:, j])
        g = np.linalg.norm(G[:, j])
        # the solve's guarantee: the residual of A^H lambda = g (rtol 1e-12 on the recursive residual), above the
        # rounding floor of forming D lambda in double precision (near a resonance ||lambda|| is large)
        floor = 64 * np.finfo(float).eps * np.linalg.norm(D) * np.linalg.norm(lam[:, j])
        assert np.linalg.norm(D @ lam[:, j] - G[:, j]) <= 1e-10 * g + floor
        # the error against the dense solve, within the conditioning: kappa >= ||A||_F ||lambda|| / ||g|| / sqrt(n)
        kest = np.linalg.norm(D) * np.linalg.norm(ld) / g / np.sqrt(A.n)
        assert np.linalg.norm(lam[:, j] - ld) / np.linalg.norm(ld) < max(1e-8, 1e-10 * kest)
        go = O.zgrad_vals(Aj, lam[:, j], X[:, j])
        assert np.max(np.abs(gv[:, j] - go)) <= 1e-14 * np.max(np.abs(go))


def test_batched_backward_equals_single_backward(hz):
    """Loss sum_j sum_r |x_j[r] - t_j[r]|^2 through helmholtz_solve_batched vs per-system helmholtz_solve."""
    B = 4
    A, vals, rhs = small_sweep(B, seed=3)
    rng = np.random.default_rng(4)
    rec = rng.choice(A.n, size=min(40, A.n), replace=False)
    T = cn(rng, len(rec), B)
    opts = hz.SolveOptions(rtol=1e-12, jacobi=True, symmetric=True)
    rp, ci = dev(A.row_ptr), dev(A.col_idx)
    V = dev(vals.T).requires_grad_(True)
    Bm = dev(rhs.T).requires_grad_(True)
    X = hz.helmholtz_solve_batched(rp, ci, V, Bm, opts)
    loss = (X[dev(rec)] - dev(T)).abs().pow(2).sum()
    loss.backward()
    for j in range(B):
        v = dev(vals[j]).requires_grad_(True)
        b = dev(rhs[j]).requires_grad_(True)
        x = hz.helmholtz_solve(rp, ci, v, b, opts)
        lj = (x[dev(rec)] - dev(T[:, j])).abs().pow(2).sum()
        lj.backward()
        gb, gv = b.grad.cpu().numpy(), v.grad.cpu().numpy()
        assert np.linalg.norm(Bm.grad[:, j].cpu().numpy() - gb) / np.linalg.norm(gb) < 1e-7
        assert np.linalg.norm(V.grad[:, j].cpu().numpy() - gv) / np.linalg.norm(gv) < 1e-7


def test_batched_adjoint_without_entry_gradients_and_statuses(hz):
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    P = CSR(rp, ci, np.zeros(4, complex))
    vals = np.array([[0, 1, 1, 0], [2, 1, 1, 3]], complex)
    G = np.array([[1, 1], [0, 1]], complex)  # column j = g_j
    lam, gv, infos = hz.zbicgstab_adjoint_batched(dev(P.row_ptr), dev(P.col_idx), dev(vals.T), None, dev(G),
                                                  rtol=1e-12, flags=hz.SYMMETRIC, want_grad_vals=False)
    assert gv is None
    assert infos[0]["status"] == hz.BREAKDOWN and infos[0]["breakdown"] == hz.BD_RHAT_V
    assert infos[1]["status"] == hz.OK
    l1 = np.linalg.solve(vals[1].reshape(2, 2).conj().T, G[:, 1])
    assert np.allclose(lam.cpu().numpy()[:, 1], l1, rtol=1e-11)
