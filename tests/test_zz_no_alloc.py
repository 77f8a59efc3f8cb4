"""The allocation-free solve (zbicgstab_solve_noalloc) against the asynchronous solve it varies.

Both run the same kernels on the same launch map.  The allocation-free call takes its workspace from the
library's static scratch and launches its iterations directly instead of replaying cached graphs; neither
changes the kernels or their order, so x and the device info must equal the asynchronous solve's bit for
bit, and the solution must meet the tolerance by the oracle's product.  Two calls in a row, the second on a
smaller system, check that what the first call leaves in the scratch does not leak into the second.  A
system whose workspace exceeds the scratch is rejected on the host before anything is enqueued.
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


def test_noalloc_equals_async_on_two_calls_second_smaller(hz):
    # first: the full cylinder under Jacobi (gather-light iteration, about 80 MB of scratch);
    # second: a 12^3 cube without preconditioner (fused iteration, a few hundred kB)
    A1, b1, _ = W.config_cylinder()
    A2, b2, _ = W.config_cube(12, seed=2)
    cases = [(A1, b1, hz.PRECOND_JACOBI, 1e-10, 3000), (A2, b2, hz.PRECOND_NONE, 1e-10, 2000)]
    outs = []
    for A, b, pre, tol, maxiter in cases:
        rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
        x = torch.full((A.n,), 7.0 + 3.0j, dtype=torch.complex128, device="cuda:0")  # ignored: X0_ZERO
        info = torch.empty(64, dtype=torch.uint8, device="cuda:0")
        xn, info_n = hz.zbicgstab_solve_noalloc(rp, ci, v, bd, x=x, rtol=tol, maxiter=maxiter,
                                                flags=pre | hz.X0_ZERO, info=info)
        torch.cuda.synchronize()
        outs.append((A, b, pre, tol, maxiter, xn.cpu().numpy(), hz.read_info(info_n)))
    for A, b, pre, tol, maxiter, xn, inf_n in outs:
        rp, ci, v, bd = dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b)
        xa, info_a = hz.zbicgstab_solve_async(rp, ci, v, bd, rtol=tol, maxiter=maxiter, flags=pre | hz.X0_ZERO)
        inf_a = hz.read_info(info_a)
        assert inf_n == inf_a, (inf_n, inf_a)
        assert np.array_equal(xn.view(np.float64), xa.cpu().numpy().view(np.float64))
        assert inf_n["status"] == hz.OK and inf_n["renumbered"] == 0
        assert true_relres(A, xn, b) <= tol * (1 + 1e-2)


def test_noalloc_rejects_systems_beyond_the_scratch(hz):
    assert hz.zbicgstab_noalloc_max_bytes() == 96 << 20
    # a valid diagonal system whose workspace (128 bytes per row without a preconditioner) exceeds 96 MiB
    n = 800_000
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda:0")
    ci = torch.arange(n, dtype=torch.int32, device="cuda:0")
    v = torch.ones(n, dtype=torch.complex128, device="cuda:0")
    b = torch.ones(n, dtype=torch.complex128, device="cuda:0")
    assert hz.zbicgstab_workspace_bytes(n, n, hz.NO_REORDER) > hz.zbicgstab_noalloc_max_bytes()
    with pytest.raises(hz.HelmzError) as e:
        hz.zbicgstab_solve_noalloc(rp, ci, v, b, rtol=1e-10, maxiter=10)
    assert e.value.code == -4
    # invalid flags are refused as for the asynchronous solve
    for bad in (hz.REORDER, hz.VALIDATE, hz.RELIABLE):
        with pytest.raises(hz.HelmzError):
            hz.zbicgstab_solve_noalloc(rp[:11], ci[:10], v[:10], b[:10], flags=bad)
