"""7-point finite-difference Helmholtz operator on a unit cube.

The continuous problem is the paper's Helmholtz equation -Lap(u) - k^2 u = g
(Section 2).  On an N x N x N grid of interior nodes with spacing
h = 1/(N+1), the h^2-scaled 7-point stencil gives

    A_ii = 6 - (k h)^2          (+ i k h beta_i on boundary rows)
    A_ij = -1                    for the in-grid axis neighbours j of i

Homogeneous Dirichlet values outside the grid are eliminated (their
couplings are dropped).  A "boundary row" is a row with at least one missing
neighbour; it receives the impedance term once, whatever the number of
missing neighbours.  ``beta`` is a per-node impedance coefficient (default
1), only read on boundary rows.

Nodes are numbered in natural order, index = (ix * N + iy) * N + iz.
"""

from __future__ import annotations

import numpy as np

from .csr import CSR, csr_from_coo


def cube_wavenumber(N: int, points_per_wavelength: float = 10.0) -> float:
    """k such that one wavelength 2*pi/k spans ``points_per_wavelength`` grid steps."""
    h = 1.0 / (N + 1)
    return 2.0 * np.pi / (points_per_wavelength * h)


def helmholtz_cube(N: int, k: float | None = None, beta: np.ndarray | None = None) -> CSR:
    if N < 1:
        raise ValueError("N must be >= 1")
    h = 1.0 / (N + 1)
    if k is None:
        k = cube_wavenumber(N)
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx // (N * N), (idx // N) % N, idx % N
    coords = (ix, iy, iz)
    strides = (N * N, N, 1)

    rows = [idx]
    cols = [idx]
    missing = np.zeros(n, dtype=bool)
    offdiag_r, offdiag_c = [], []
    for axis in range(3):
        c = coords[axis]
        for sgn in (-1, 1):
            ok = (c + sgn >= 0) & (c + sgn < N)
            missing |= ~ok
            offdiag_r.append(idx[ok])
            offdiag_c.append(idx[ok] + sgn * strides[axis])
    rows += offdiag_r
    cols += offdiag_c

    if beta is None:
        beta = np.ones(n, dtype=np.complex128)
    beta = np.asarray(beta, dtype=np.complex128)
    if beta.shape != (n,):
        raise ValueError("beta must have one entry per node")
    kh = k * h
    diag = np.full(n, 6.0 - kh * kh, dtype=np.complex128)
    diag[missing] += 1j * kh * beta[missing]
    n_off = sum(a.size for a in offdiag_r)
    vals = np.concatenate([diag, np.full(n_off, -1.0 + 0.0j)])

    A = csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), vals)
    A.meta = {
        "kind": "cube7",
        "N": N,
        "h": h,
        "k": float(k),
        "boundary_rows": np.flatnonzero(missing),
        "interior_rows": np.flatnonzero(~missing),
        "grid": (N, N, N),
    }
    return A


def cube_node_coords(N: int) -> np.ndarray:
    """Physical coordinates (n, 3) of the interior grid nodes, spacing 1/(N+1)."""
    h = 1.0 / (N + 1)
    idx = np.arange(N * N * N, dtype=np.int64)
    ix, iy, iz = idx // (N * N), (idx // N) % N, idx % N
    return np.stack([(ix + 1) * h, (iy + 1) * h, (iz + 1) * h], axis=1)
