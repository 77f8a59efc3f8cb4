"""Invariants of the synthetic input generators (no solver arithmetic)."""

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from workloads.fem import _tet_local, assemble_helmholtz_p1, cylinder_mesh, cabin_mesh
from workloads.rng import make_rng


def _sp(A, vals=None):
    return sp.csr_matrix((A.vals if vals is None else vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))


def test_cube_sizes_and_symmetry():
    A, b, info = W.config_cube(20)
    A.check()
    assert A.n == 8000 and A.nnz == 8000 + 6 * 19 * 20 * 20 == 53600
    S = _sp(A)
    assert (S != S.T).nnz == 0
    h, k = A.meta["h"], A.meta["k"]
    assert h == 1 / 21 and abs(k * h - 2 * np.pi / 10) < 1e-15
    d = S.diagonal()
    inter = A.meta["interior_rows"]
    bnd = A.meta["boundary_rows"]
    assert np.all(d[inter] == 6 - (k * h) ** 2)
    assert np.allclose(d[bnd].imag, k * h, rtol=0, atol=1e-15)
    assert inter.size == 18**3
    # right-hand side: one unit source at an interior node plus small noise
    big = np.flatnonzero(np.abs(b) > 0.5)
    assert big.size == 1 and big[0] in set(inter.tolist())
    assert 0.5e-3 < np.std(b.real[np.abs(b) < 0.5]) < 2e-3


def test_cube_is_seeded():
    _, b0, _ = W.config_cube(6, seed=11)
    _, b1, _ = W.config_cube(6, seed=11)
    _, b2, _ = W.config_cube(6, seed=12)
    assert np.array_equal(b0, b1) and not np.array_equal(b0, b2)


@pytest.mark.parametrize("robin", ["caps", "all"])
def test_small_cylinder_fem_invariants(robin):
    rng = make_rng(0)
    h = 0.125
    mesh = cylinder_mesh(h=h, rng=rng, robin=robin)
    vol, _ = _tet_local(mesh["coords"], mesh["tets"])
    assert np.all(vol > 0)
    assert abs(vol.sum() - mesh["n_cubes"] * h**3) < 1e-12 * mesh["n_cubes"] * h**3
    asm = assemble_helmholtz_p1(mesh, 2.0, mesh["robin_sel"])
    A = asm["A"]
    A.check()
    ones = np.ones(A.n)
    K, M, B = _sp(A, asm["K"]), _sp(A, asm["M"]), _sp(A, asm["B"])
    # bitwise symmetry of every part and of A
    for X in (K, M, B, _sp(A)):
        assert (X != X.T).nnz == 0
    # constants are in the stiffness kernel; mass sums to the volume
    assert np.max(np.abs(K @ ones)) < 1e-12
    assert abs(ones @ (M @ ones) - vol.sum()) < 1e-12
    # boundary mass sums to the area of the Robin squares (boundary nodes are not jittered)
    area = mesh["robin_sel"].sum() * h * h
    assert abs(ones @ (B @ ones) - area) < 1e-12 * max(1, area)
    # values: A = K - k^2 M + i k B
    assert np.array_equal(A.vals, (asm["K"] - 4.0 * asm["M"]) + 1j * (2.0 * asm["B"]))
    # Kuhn pattern: at most 15 entries per row, diagonal present
    lens = np.diff(A.row_ptr)
    assert lens.max() == 15
    S = _sp(A)
    assert np.all(S.diagonal() != 0)


def test_cylinder_default_sizes():
    A, b, info = W.config_cylinder()
    assert A.n == 209777 and A.nnz == 3048433
    assert (lambda s: (s != s.T).nnz)(_sp(A)) == 0


def test_cabin_small_permuted():
    A, b, info = W.config_cabin(h=0.1, k=5.0, seed=3)
    A.check()
    perm = info["perm"]
    assert np.array_equal(np.sort(perm), np.arange(A.n))
    S = _sp(A)
    assert (S != S.T).nnz == 0
    A0, b0, _ = W.config_cabin(h=0.1, k=5.0, seed=3, permute=False)
    S0 = _sp(A0)
    # P A0 P^T == A
    P = sp.csr_matrix((np.ones(A.n), (perm, np.arange(A.n))), shape=(A.n, A.n))
    assert abs(P @ S0 @ P.T - S).max() == 0


def test_freq_sweep_shares_pattern():
    A, vals, rhs, ks, info = W.config_freq_sweep(B=3, h=0.25)
    assert vals.shape == (3, A.nnz) and rhs.shape == (3, A.n)
    assert np.all((ks >= 10) & (ks <= 40))


def test_cube_batch_sizes():
    systems, info = W.config_cube_batch(B=4, nmin=4, nmax=7)
    assert [A.n for A, _ in systems] == [N**3 for N in info["Ns"]]


def test_impedance_maps_reproduce_boundary_terms():
    """Phi beta with beta = 1 equals the impedance part of the assembled matrix."""
    A, _, _ = W.config_cube(8)
    m = W.cube_impedance_map(A)
    rp, ci, v = m["phi"]
    Phi = sp.csr_matrix((v, ci, rp), shape=m["shape"])
    d = Phi @ np.ones(A.n)
    assert np.array_equal(d.imag != 0, np.isin(np.arange(A.nnz), W.entry_positions(A, A.meta["boundary_rows"], A.meta["boundary_rows"])))
    assert np.allclose(d[d != 0], 1j * A.meta["k"] * A.meta["h"])
    A, _, info = W.config_cylinder(h=0.25, k=3.0, with_parts=True)
    asm = info["parts"]
    m = W.fem_impedance_map(A, asm["tris"], A.meta["coords"], 3.0)
    rp, ci, v = m["phi"]
    Phi = sp.csr_matrix((v, ci, rp), shape=m["shape"])
    assert np.max(np.abs(Phi @ np.ones(A.n) - 1j * 3.0 * asm["B"])) < 1e-15
    rp2, ci2, v2 = m["phi_h"]
    assert abs(sp.csr_matrix((v2, ci2, rp2), shape=(A.n, A.nnz)) - Phi.conj().T).max() == 0
