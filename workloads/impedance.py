"""Matrix entries as an affine function of per-node impedance coefficients.

The Helmholtz matrices here are affine in a per-node impedance coefficient
beta (default 1 everywhere):  vals(beta) = vals_rest + Phi beta, with Phi a
sparse (nnz x n) complex matrix.  These builders return Phi and Phi^H in
CSR so that gradients with respect to the matrix entries can be chained to
beta.  They only describe how the inputs are assembled (no solver
arithmetic).

cube (7-point FD): a boundary row i carries + i k h beta_i on its diagonal,
    so Phi[p(i,i), i] = i k h.
P1 FEM: B(beta)_ij = sum_m beta_m int_F phi_m phi_i phi_j over the Robin
    faces F, with the exact P1 face integrals |F|/10 (i = j = m), |F|/30
    (two of i, j, m equal) and |F|/60 (all distinct); A carries i k B(beta),
    so Phi[p(i,j), m] = i k sum_F |F| c(i,j,m).  With beta = 1 this is
    i k B, B the Robin boundary mass.
"""

from __future__ import annotations

import numpy as np


def entry_positions(A, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """CSR positions of entries (rows[k], cols[k]); every entry must exist."""
    n = A.n
    keys = A.row_of_entry() * n + A.col_idx.astype(np.int64)  # sorted: rows, then columns
    q = rows.astype(np.int64) * n + cols.astype(np.int64)
    pos = np.searchsorted(keys, q)
    if np.any(pos >= keys.size) or np.any(keys[np.minimum(pos, keys.size - 1)] != q):
        raise ValueError("entry not in the sparsity pattern")
    return pos


def _coo_to_csr(nrows: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    key = rows.astype(np.int64) * (int(cols.max()) + 1 if cols.size else 1) + cols.astype(np.int64)
    uk, inv = np.unique(key, return_inverse=True)
    summed = np.zeros(uk.size, dtype=np.complex128)
    np.add.at(summed, inv, vals)
    ncol = int(cols.max()) + 1 if cols.size else 1
    r = (uk // ncol).astype(np.int64)
    c = (uk % ncol).astype(np.int64)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=nrows), out=rp[1:])
    return rp.astype(np.int32), c.astype(np.int32), summed


def _phi_pair(nnz: int, n: int, p: np.ndarray, m: np.ndarray, v: np.ndarray):
    """CSR of Phi (nnz x n) and Phi^H (n x nnz) from COO triplets (p, m, v)."""
    phi = _coo_to_csr(nnz, p, m, v)
    phi_h = _coo_to_csr(n, m, p, np.conj(v))
    return {"phi": phi, "phi_h": phi_h, "shape": (nnz, n)}


def cube_impedance_map(A) -> dict:
    h, k = A.meta["h"], A.meta["k"]
    rows = np.asarray(A.meta["boundary_rows"], dtype=np.int64)
    p = entry_positions(A, rows, rows)
    return _phi_pair(A.nnz, A.n, p, rows, np.full(rows.size, 1j * k * h))


def fem_impedance_map(A, tris: np.ndarray, coords: np.ndarray, k: float) -> dict:
    """Phi for P1 elements; ``tris`` are the Robin triangles (node ids)."""
    X = coords[tris]
    area = 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1)
    P, M, V = [], [], []
    for a in range(3):
        for b in range(3):
            for m in range(3):
                same = (a == b) + (b == m) + (a == m)
                c = 1.0 / 10.0 if same == 3 else (1.0 / 30.0 if same == 1 else 1.0 / 60.0)
                P.append(entry_positions(A, tris[:, a], tris[:, b]))
                M.append(tris[:, m])
                V.append(1j * k * c * area)
    return _phi_pair(A.nnz, A.n, np.concatenate(P), np.concatenate(M), np.concatenate(V))
