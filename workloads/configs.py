"""Seeded builders for the benchmark and test workloads.

Each builder returns plain numpy arrays.  One ``numpy.random.default_rng``
stream per builder is consumed in a fixed, documented order, so a seed
names an input exactly.

Workloads
---------
cube      7-point FD Helmholtz on an N^3 grid (default N = 20, n = 8000),
          k for 10 points per wavelength, impedance on boundary rows.
cylinder  P1 Kuhn-tetrahedral FEM on a cylinder of radius 1 and length 4
          (default h = 0.04: about 2.1e5 nodes, 3.0e6 non-zeros), k = 20,
          Robin (impedance) end caps and, by default, lateral wall.
cabin     P1 FEM on a 2.0 x 1.2 x 1.1 box with two seat cut-outs
          (default h = 0.012: about 1.2e6 nodes, 1.8e7 non-zeros), k = 40,
          Robin outer walls, node numbering randomly permuted.
freq      one cylinder pattern with B frequencies k ~ U(10, 40).
cubes     B independent cubes with N ~ U{16..64}, each with its own k.
adjoint   cylinder with receivers, targets and point sources for a
          least-squares loss.

The right-hand side of a single solve is a unit point source at a seeded
interior node plus complex Gaussian noise whose real and imaginary parts
each have standard deviation 1e-3.
"""

from __future__ import annotations

import numpy as np

from .csr import CSR, permute_symmetric
from .cube import cube_node_coords, cube_wavenumber, helmholtz_cube
from .fem import assemble_helmholtz_p1, cabin_mesh, cylinder_mesh
from .rng import cn_vector, make_rng

NOISE_STD = 1e-3


def point_source_rhs(n: int, interior: np.ndarray, rng: np.random.Generator, noise_std: float = NOISE_STD):
    """Unit source at ``interior[rng.integers(len(interior))]`` plus noise.

    Draw order: the node index, then the n real parts, then the n imaginary
    parts of the noise.
    """
    node = int(interior[rng.integers(interior.shape[0])])
    b = cn_vector(rng, n, std=noise_std)
    b[node] += 1.0
    return b, node


def plane_wave(coords: np.ndarray, kappa: float, axis: int = 0) -> np.ndarray:
    """u_j = exp(i kappa x_j) along one coordinate axis."""
    return np.exp(1j * kappa * coords[:, axis]).astype(np.complex128)


def csr_example_arrays():
    """The 5 x 5 real matrix of the paper's CSR illustration (Section 3.2), 0-based."""
    row_ptr = np.array([0, 2, 4, 6, 9, 11], dtype=np.int32)
    col_idx = np.array([0, 1, 1, 2, 0, 2, 1, 3, 4, 2, 4], dtype=np.int32)
    vals = np.array([3, 14, 8, 1, 2, 6, 4, 2, -1, 9, 7], dtype=np.complex128)
    return row_ptr, col_idx, vals


def csr_example() -> CSR:
    rp, ci, v = csr_example_arrays()
    return CSR(rp, ci, v, {"kind": "paper_example"})


def config_cube(N: int = 20, seed: int = 0, k: float | None = None):
    """7-point cube; returns (A, b, info)."""
    A = helmholtz_cube(N, k=k)
    rng = make_rng(seed)
    b, node = point_source_rhs(A.n, A.meta["interior_rows"], rng)
    A.meta["coords"] = cube_node_coords(N)
    return A, b, {"source_node": node, "seed": seed, "workload": f"cube7_N{N}"}


def _fem_rhs(mesh, A: CSR, rng):
    interior = np.flatnonzero(~mesh["boundary_node"])
    return point_source_rhs(A.n, interior, rng)


def config_cylinder(
    h: float = 0.04, k: float = 20.0, seed: int = 0, jitter: float = 0.1, with_parts: bool = False, robin: str = "all"
):
    """Cylinder FEM; draw order: node jitter, then the right-hand side."""
    rng = make_rng(seed)
    mesh = cylinder_mesh(h=h, rng=rng, jitter=jitter, robin=robin)
    asm = assemble_helmholtz_p1(mesh, k, mesh["robin_sel"])
    A = asm["A"]
    A.meta["coords"] = mesh["coords"]
    b, node = _fem_rhs(mesh, A, rng)
    info = {"source_node": node, "seed": seed, "workload": f"cylinder_h{h:g}_k{k:g}", "mesh": mesh}
    if with_parts:
        info["parts"] = asm
    return A, b, info


def config_cabin(h: float = 0.012, k: float = 40.0, seed: int = 0, permute: bool = True, jitter: float = 0.1):
    """Cabin FEM; draw order: seats, jitter, node permutation, right-hand side.

    With ``permute`` the returned system is P A P^T x' = P b; ``info["perm"]``
    maps an original node ``i`` to its new index ``perm[i]``.
    """
    rng = make_rng(seed)
    mesh = cabin_mesh(h=h, rng=rng, jitter=jitter)
    asm = assemble_helmholtz_p1(mesh, k, mesh["robin_sel"])
    A = asm["A"]
    n = A.n
    perm = rng.permutation(n)  # drawn either way, so both numberings share the right-hand side
    if not permute:
        perm = np.arange(n)
    interior = np.flatnonzero(~mesh["boundary_node"])
    b, node = point_source_rhs(n, interior, rng)
    if permute:
        A = permute_symmetric(A, perm)
        bp = np.empty_like(b)
        bp[perm] = b
        b = bp
    A.meta.update({"kind": "p1", "k": float(k), "h": float(h)})
    coords = np.empty_like(mesh["coords"])
    coords[perm] = mesh["coords"]
    A.meta["coords"] = coords
    info = {"source_node": int(perm[node]), "seed": seed, "perm": perm, "workload": f"cabin_h{h:g}_k{k:g}"}
    return A, b, info


def config_freq_sweep(
    B: int = 64, h: float = 0.04, seed: int = 0, kmin: float = 10.0, kmax: float = 40.0, robin: str = "all"
):
    """B Helmholtz systems A(k_j) = K - k_j^2 M + i k_j B on one cylinder pattern.

    Draw order: node jitter, the B wavenumbers, then B right-hand sides
    (each drawn as in a single solve).  Returns (pattern CSR with the first
    system's values, vals (B, nnz), rhs (B, n), ks, info); info["K"],
    info["M"], info["B"] are the real matrices on the pattern.
    """
    rng = make_rng(seed)
    mesh = cylinder_mesh(h=h, rng=rng, robin=robin)
    asm = assemble_helmholtz_p1(mesh, 1.0, mesh["robin_sel"])
    K, M, Bm = asm["K"], asm["M"], asm["B"]
    ks = rng.uniform(kmin, kmax, size=B)
    vals = np.empty((B, K.shape[0]), dtype=np.complex128)
    for j, kj in enumerate(ks):
        vals[j] = (K - (kj * kj) * M) + 1j * (kj * Bm)
    interior = np.flatnonzero(~mesh["boundary_node"])
    A = asm["A"].with_vals(vals[0])
    rhs = np.stack([point_source_rhs(A.n, interior, rng)[0] for _ in range(B)])
    return A, vals, rhs, ks, {"seed": seed, "workload": f"freq_sweep_B{B}_h{h:g}", "K": K, "M": M, "B": Bm}


def config_cube_batch(B: int = 32, seed: int = 0, nmin: int = 16, nmax: int = 64):
    """B independent cubes with N_j ~ U{nmin..nmax} and k_j for 10 points per wavelength.

    Draw order: the B sizes, then for each cube in turn its right-hand side.
    """
    rng = make_rng(seed)
    Ns = rng.integers(nmin, nmax + 1, size=B)
    systems = []
    for N in Ns:
        A = helmholtz_cube(int(N), k=cube_wavenumber(int(N)))
        b, _ = point_source_rhs(A.n, A.meta["interior_rows"], rng)
        systems.append((A, b))
    return systems, {"seed": seed, "Ns": Ns.tolist(), "workload": f"cube_batch_B{B}"}


def config_adjoint(
    h: float = 0.04,
    k: float = 20.0,
    seed: int = 0,
    n_receivers: int = 1000,
    n_sources: int = 50,
    jitter: float = 0.1,
    robin: str = "all",
):
    """Least-squares inverse-problem inputs on the cylinder.

    Draw order: node jitter, receiver nodes, target values, source nodes,
    source amplitudes.  The loss is L = sum_r |x_r - t_r|^2 with
    b = sum_s a_s e_s.
    """
    rng = make_rng(seed)
    mesh = cylinder_mesh(h=h, rng=rng, jitter=jitter, robin=robin)
    asm = assemble_helmholtz_p1(mesh, k, mesh["robin_sel"])
    A = asm["A"]
    n = A.n
    receivers = rng.choice(n, size=n_receivers, replace=False)
    targets = cn_vector(rng, n_receivers)
    sources = rng.choice(n, size=n_sources, replace=False)
    amps = cn_vector(rng, n_sources)
    return A, {
        "receivers": receivers,
        "targets": targets,
        "sources": sources,
        "amps": amps,
        "parts": asm,
        "mesh": mesh,
        "seed": seed,
        "workload": f"adjoint_cylinder_h{h:g}_k{k:g}",
    }
