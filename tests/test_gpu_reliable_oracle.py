"""GPU parity of the reliable-update mixed-precision solve against its oracle (oracle/reliable.py).

Both run Jacobi- or un-preconditioned BiCGStab in complex64 on A D^{-1} y = b / ||b|| with reliable updates
each time the recursive residual has fallen tenfold (delta = 0.1), and decide convergence on the complex128
true residual.  Unique: the tolerance met by the true residual (recomputed with the oracle's complex128 SpMV)
and the solution, up to the conditioning (both within 1e-8 of a complex128 solve to 1e-13; the oracle's own
distance is about 3e-10 on these systems).  Not unique: the iteration and update counts, which depend on the
order of the complex64 sums; they are checked to lie within a factor of two of the oracle's.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle.reliable import zbicgstab_reliable

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def case(name):
    if name == "cube20":  # the 20^3 finite-difference cube, unpreconditioned
        A, b, _ = W.config_cube()
        return A, b, False
    F, vals, rhs, ks, _ = W.config_freq_sweep(B=1, h=0.12, kmin=5.0, kmax=5.0, seed=3)  # P1 cylinder, Jacobi
    return F.with_vals(vals[0]), rhs[0], True


@pytest.mark.parametrize("name", ["cube20", "fem"])
def test_reliable_updates_match_the_oracle(hz, name):
    A, b, jacobi = case(name)
    xo, io = zbicgstab_reliable(A, b, tol=1e-10, delta=0.1, jacobi=jacobi)
    xr, ir = O.zbicgstab(A, b, tol=1e-13, maxiter=50000, jacobi=jacobi)
    assert io["status"] == 0 and ir["status"] == 0
    flags = hz.X0_ZERO | hz.RELIABLE | (hz.PRECOND_JACOBI if jacobi else 0)
    x, info = hz.zbicgstab_solve_mixed(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(b), rtol=1e-10,
                                       inner_rtol=0.1, maxiter=50000, flags=flags)
    assert info["status"] == hz.OK, info
    x = x.cpu().numpy()
    rr = np.linalg.norm(b - O.zspmv(A, x)) / np.linalg.norm(b)
    assert rr <= 1e-10 * (1 + 1e-3)
    nr = np.linalg.norm(xr)
    assert np.linalg.norm(x - xr) / nr < 1e-8
    assert np.linalg.norm(xo - xr) / nr < 1e-8
    assert np.linalg.norm(x - xo) / nr < 2e-8
    assert 0.5 <= info["iterations"] / io["iterations"] <= 2.0, (info, io)
    assert info["outer_steps"] >= 2 and io["outer_steps"] >= 2
    print(f"{name}: GPU {info['iterations']} iterations / {info['outer_steps']} updates, "
          f"oracle {io['iterations']} / {io['outer_steps']}, relres {rr:.2e}")
