"""Solver iterations replayed from captured HIP graphs.

Every solver enqueues its iterations in chunks; each chunk is captured once
into a graph cached in the handle and replayed by one hipGraphLaunch.  The
kernels and their order are those of the direct launches, so a solve with
graphs must equal, bitwise, the same solve with HZ_NO_GRAPH=1 (direct
launches), on every replay of a cached graph, with other eager GPU work and
synchronisations between the replays, and after the cache has evicted
entries.
"""

import os

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


def bits(t):
    return t.detach().cpu().numpy().view(np.float64).copy()


def eager(fn):
    os.environ["HZ_NO_GRAPH"] = "1"
    try:
        return fn()
    finally:
        del os.environ["HZ_NO_GRAPH"]


def other_work(hz, k):
    """Eager GPU work between replays: a product, torch arithmetic, a sync."""
    A, _, _ = W.config_cube(6, seed=k)
    y = hz.csr_zspmv(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(np.ones(A.n, complex)))
    z = (y * (1 + 1j)).sum()
    torch.cuda.synchronize()
    return complex(z.item())


def test_single_solve_replays_equal_direct_launches(hz):
    A, b, _ = W.config_cube(14, seed=1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    ws = hz.workspace(A.n, A.nnz, hz.PRECOND_NONE | hz.X0_ZERO, "cuda:0")
    x = torch.zeros(A.n, dtype=torch.complex128, device="cuda:0")
    xe, ie = eager(lambda: hz.zbicgstab_solve(rp, ci, v, bd, x=x.clone(), rtol=1e-10, ws=ws))
    ref = bits(xe)
    for k in range(4):  # the first call captures, the others replay the cached graphs
        xg, ig = hz.zbicgstab_solve(rp, ci, v, bd, x=x.clone(), rtol=1e-10, ws=ws)
        assert ig == ie
        assert np.array_equal(bits(xg), ref)
        other_work(hz, k)
    assert ie["status"] == hz.OK
    assert np.linalg.norm(b - O.zspmv(A, xe.cpu().numpy())) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-3)


def test_jacobi_solve_with_tail_chunk_and_not_converged(hz):
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    ws = hz.workspace(A.n, A.nnz, flags, "cuda:0")
    for maxiter in (37, 37, 5000):  # 37 = 8 + 16 + 13: a partial last chunk and the concluding kernel
        xe, ie = eager(lambda: hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, maxiter=maxiter, flags=flags, ws=ws))
        xg, ig = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, maxiter=maxiter, flags=flags, ws=ws)
        assert ig == ie and np.array_equal(bits(xg), bits(xe))
        other_work(hz, maxiter)
    assert ie["status"] == hz.OK
    ig37 = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, maxiter=37, flags=flags, ws=ws)[1]
    assert ig37["status"] == hz.NOT_CONVERGED and ig37["iterations"] == 37


def test_varbatch_and_shared_pattern_batches_replay_equal(hz):
    systems, _ = W.config_cube_batch(B=6, nmin=5, nmax=12, seed=4)
    row_off = np.concatenate([[0], np.cumsum([A.n for A, _ in systems])]).astype(np.int32)
    nnz_off = np.concatenate([[0], np.cumsum([A.nnz for A, _ in systems])])
    rp = np.concatenate([A.row_ptr[:-1] + nnz_off[j] for j, (A, _) in enumerate(systems)] + [nnz_off[-1:]])
    ci = np.concatenate([A.col_idx.astype(np.int64) + row_off[j] for j, (A, _) in enumerate(systems)])
    vals = np.concatenate([A.vals for A, _ in systems])
    b = np.concatenate([bb for _, bb in systems])
    args = (row_off, dev(rp.astype(np.int32)), dev(ci.astype(np.int32)), dev(vals), dev(b))
    xe, ie = eager(lambda: hz.zbicgstab_solve_varbatch(*args, rtol=1e-10))
    for k in range(3):
        xg, ig = hz.zbicgstab_solve_varbatch(*args, rtol=1e-10)
        assert ig == ie and np.array_equal(bits(xg), bits(xe))
        other_work(hz, k)
    A, vals, rhs, ks, info = W.config_freq_sweep(B=5, h=0.15, kmin=3.0, kmax=6.0, seed=2)
    margs = (dev(A.row_ptr), dev(A.col_idx), dev(vals.T), dev(rhs.T))
    xe, ie = eager(lambda: hz.zbicgstab_solve_batched(*margs, rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.X0_ZERO))
    sargs = (dev(A.row_ptr), dev(A.col_idx), dev(info["K"]), dev(info["M"]), dev(info["B"]), ks, dev(rhs.T))
    se, sie = eager(lambda: hz.zbicgstab_solve_sweep(*sargs, rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.X0_ZERO))
    for k in range(3):
        xg, ig = hz.zbicgstab_solve_batched(*margs, rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
        assert ig == ie and np.array_equal(bits(xg), bits(xe))
        sg, sig = hz.zbicgstab_solve_sweep(*sargs, rtol=1e-10, flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
        assert sig == sie and np.array_equal(bits(sg), bits(se))
        other_work(hz, k)
    assert all(i["status"] == hz.OK for i in ie + sie)


@pytest.mark.parametrize("reliable", [False, True])
def test_mixed_solves_replay_equal(hz, reliable):
    A, b, _ = W.config_cylinder(h=0.1)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO | (hz.RELIABLE if reliable else 0)
    ws = hz.mixed_workspace(A.n, A.nnz, flags, "cuda:0")
    xe, ie = eager(lambda: hz.zbicgstab_solve_mixed(rp, ci, v, bd, rtol=1e-10, flags=flags, ws=ws))
    for k in range(3):
        xg, ig = hz.zbicgstab_solve_mixed(rp, ci, v, bd, rtol=1e-10, flags=flags, ws=ws)
        assert ig == ie and np.array_equal(bits(xg), bits(xe))
        other_work(hz, k)
    assert ie["status"] == hz.OK


def test_graph_cache_eviction_keeps_results(hz):
    """More distinct chunk graphs than the cache holds (32): evicted entries are re-captured."""
    A, b, _ = W.config_cube(10, seed=2)
    rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
    xe, ie = eager(lambda: hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10))
    wss = [hz.workspace(A.n, A.nnz, hz.X0_ZERO, "cuda:0") for _ in range(12)]  # new pointers: new keys
    for rnd in range(2):
        for ws in wss:
            xg, ig = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, ws=ws)
            assert ig == ie and np.array_equal(bits(xg), bits(xe))
