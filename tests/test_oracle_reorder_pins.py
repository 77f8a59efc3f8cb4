"""Pins of the oracle's level-set ordering and symmetric permutation.

The ordering has a plain definition (graph distances from a start found by
one pseudo-peripheral step, then Cuthill-McKee within the levels); these tests fix
it by closed forms on graphs whose distances are known (paths, grids, cubes),
by the defining properties of breadth-first levels on a scrambled mesh, by
equality with the textbook queue form of Cuthill-McKee, and by an
independent route to P A P^T (dense permutation, COO re-sort).
"""

import numpy as np
import pytest

import oracle.reorder as R
import workloads as W
from workloads.csr import CSR, csr_from_coo, permute_symmetric


def path_csr(n):
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    return csr_from_coo(n, np.array(rows), np.array(cols), np.arange(1, len(rows) + 1).astype(np.complex128))


def grid_csr(nx, ny):
    idx = lambda x, y: x + nx * y  # noqa: E731
    rows, cols = [], []
    for y in range(ny):
        for x in range(nx):
            for dx, dy in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= x + dx < nx and 0 <= y + dy < ny:
                    rows.append(idx(x, y))
                    cols.append(idx(x + dx, y + dy))
    return csr_from_coo(nx * ny, np.array(rows), np.array(cols), np.ones(len(rows), np.complex128))


def test_path_graph_closed_form():
    n = 50
    A = path_csr(n)
    perm, inv, level = R.level_order(A.row_ptr, A.col_idx)
    # from node 0 the deepest node is n-1; from there level(i) = n-1-i
    assert np.array_equal(level, n - 1 - np.arange(n))
    assert np.array_equal(perm, np.arange(n)[::-1])
    assert np.array_equal(inv[perm], np.arange(n))


def textbook_cuthill_mckee(row_ptr, col_idx, start):
    """Queue form: take nodes in order, append each one's unvisited neighbours by (degree, index)."""
    n = len(row_ptr) - 1
    deg = np.diff(row_ptr)
    seen = np.zeros(n, bool)
    seen[start] = True
    order, head = [start], 0
    while head < len(order):
        v = order[head]
        head += 1
        new = sorted({int(c) for c in col_idx[row_ptr[v]:row_ptr[v + 1]] if not seen[c]}, key=lambda c: (deg[c], c))
        for c in new:
            seen[c] = True
        order.extend(new)
    return np.array(order)


def test_grid_levels_are_manhattan_distances_from_far_corner():
    nx, ny = 9, 6
    A = grid_csr(nx, ny)
    perm, inv, level = R.level_order(A.row_ptr, A.col_idx)
    x, y = np.arange(nx * ny) % nx, np.arange(nx * ny) // nx
    assert np.array_equal(level, (nx - 1 - x) + (ny - 1 - y))
    assert perm[0] == nx * ny - 1 and np.all(np.diff(level[perm]) >= 0)


@pytest.mark.parametrize("case", ["grid", "cube", "scrambled_cube", "random_graph"])
def test_level_formulation_equals_textbook_cuthill_mckee(case):
    rng = np.random.default_rng(11)
    if case == "grid":
        A = grid_csr(7, 5)
    elif case == "cube":
        A = W.helmholtz_cube(5)
    elif case == "scrambled_cube":
        A0 = W.helmholtz_cube(6)
        A = permute_symmetric(A0, rng.permutation(A0.n))
    else:  # connected random graph: a path plus random symmetric chords, varied degrees
        n = 300
        r = np.concatenate([np.arange(n - 1), rng.integers(0, n, 400)])
        c = np.concatenate([np.arange(1, n), rng.integers(0, n, 400)])
        keep = r != c
        r, c = r[keep], c[keep]
        rows = np.concatenate([r, c, np.arange(n)])
        cols = np.concatenate([c, r, np.arange(n)])
        key = np.unique(rows * n + cols)
        A = csr_from_coo(n, key // n, key % n, np.ones(key.size, complex))
    perm, inv, level = R.level_order(A.row_ptr, A.col_idx)
    assert np.array_equal(perm, textbook_cuthill_mckee(A.row_ptr, A.col_idx, int(perm[0])))
    assert np.array_equal(inv[perm], np.arange(A.n))


def test_cube_levels_are_3d_manhattan_distances():
    N = 5
    A = W.helmholtz_cube(N)
    _, _, level = R.level_order(A.row_ptr, A.col_idx)
    i = np.arange(N**3)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    assert np.array_equal(level, (N - 1 - x) + (N - 1 - y) + (N - 1 - z))


def test_unreached_component_goes_last_in_index_order():
    a, b = path_csr(7), path_csr(5)
    # component b first in the numbering, then a: node 0 lies in b
    rp = np.concatenate([b.row_ptr[:-1], a.row_ptr + b.nnz]).astype(np.int32)
    ci = np.concatenate([b.col_idx, a.col_idx + b.n]).astype(np.int32)
    A = CSR(rp, ci, np.concatenate([b.vals, a.vals]))
    perm, inv, level = R.level_order(A.row_ptr, A.col_idx)
    assert np.array_equal(level[:5], 4 - np.arange(5))
    assert np.all(level[5:] == -1)
    assert np.array_equal(perm, np.concatenate([np.arange(5)[::-1], 5 + np.arange(7)]))


def test_single_node():
    perm, inv, level = R.level_order(np.array([0, 1]), np.array([0]))
    assert list(perm) == [0] and list(inv) == [0] and list(level) == [0]


def test_scrambled_mesh_levels_have_the_breadth_first_properties():
    A, _, _ = W.config_cube(9, seed=1)
    rng = np.random.default_rng(3)
    A = permute_symmetric(A, rng.permutation(A.n))
    perm, inv, level = R.level_order(A.row_ptr, A.col_idx)
    rows = A.row_of_entry()
    cols = A.col_idx.astype(np.int64)
    assert np.all(np.abs(level[rows] - level[cols]) <= 1)  # edges join equal or adjacent levels
    assert np.count_nonzero(level == 0) == 1 and perm[0] == np.flatnonzero(level == 0)[0]
    # every node past level 0 has a neighbour one level closer
    closer = np.zeros(A.n, bool)
    closer[rows[level[cols] == level[rows] - 1]] = True
    assert np.all(closer[level > 0])
    # the renumbered matrix is banded: no entry farther than two level widths
    width = np.bincount(level).max()
    assert np.abs(inv[rows] - inv[cols]).max() <= 2 * width


def test_permute_matches_dense_and_coo_routes():
    A, _, _ = W.config_cube(5, seed=2)
    rng = np.random.default_rng(7)
    A = permute_symmetric(A, rng.permutation(A.n))
    A = CSR(A.row_ptr, A.col_idx, A.vals * (1 + 0.25j * np.arange(A.nnz)))  # distinct values
    perm, inv, _ = R.level_order(A.row_ptr, A.col_idx)
    rp, ci, v = R.permute(A.row_ptr, A.col_idx, A.vals, perm, inv)
    D = np.zeros((A.n, A.n), complex)
    D[A.row_of_entry(), A.col_idx] = A.vals
    B = np.zeros((A.n, A.n), complex)
    B[np.repeat(np.arange(A.n), np.diff(rp)), ci] = v
    assert np.array_equal(B, D[np.ix_(perm, perm)])
    Q = permute_symmetric(A, inv)  # renumber old i as inv[i], via a COO sort
    assert np.array_equal(rp, Q.row_ptr) and np.array_equal(ci, Q.col_idx) and np.array_equal(v, Q.vals)
    assert all(np.all(np.diff(ci[rp[k]:rp[k + 1]]) > 0) for k in range(A.n))
