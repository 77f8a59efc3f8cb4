"""Seeded synthetic inputs for the Helmholtz Krylov path.

This package only *builds inputs*: sparse Helmholtz matrices in CSR form
(a 7-point finite-difference cube and P1 tetrahedral finite elements on
cylinder- and cabin-shaped domains), right-hand sides and random vectors.
It carries none of the solver arithmetic (no SpMV, dot products, vector
updates or Krylov iterations), so that both the CPU oracle and the GPU path
can consume it without sharing any code of the method.

All arrays follow the paper's CSR description (Section 3.2), made 0-based:
``row_ptr`` int32[n+1], ``col_idx`` int32[nnz] sorted within each row with
the diagonal present, and ``vals`` complex128[nnz] holding interleaved
(re, im) pairs, the layout of the paper's complex structure (Section 4).
"""

from .csr import CSR
from .rng import cn_vector, make_rng
from .cube import helmholtz_cube, cube_wavenumber
from .fem import kuhn_mesh, assemble_helmholtz_p1, cylinder_mesh, cabin_mesh
from .impedance import cube_impedance_map, fem_impedance_map, entry_positions
from .configs import (
    csr_example,
    config_cube,
    config_cylinder,
    config_cabin,
    config_freq_sweep,
    config_cube_batch,
    config_adjoint,
    point_source_rhs,
    plane_wave,
)

__all__ = [
    "CSR",
    "cn_vector",
    "make_rng",
    "helmholtz_cube",
    "cube_wavenumber",
    "kuhn_mesh",
    "assemble_helmholtz_p1",
    "cylinder_mesh",
    "cabin_mesh",
    "cube_impedance_map",
    "fem_impedance_map",
    "entry_positions",
    "csr_example",
    "config_cube",
    "config_cylinder",
    "config_cabin",
    "config_freq_sweep",
    "config_cube_batch",
    "config_adjoint",
    "point_source_rhs",
    "plane_wave",
]
