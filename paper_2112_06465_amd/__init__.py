"""helmz: complex-double BiCGStab for sparse Helmholtz systems on MI355X.

The compute path is the C-ABI library ``libhelmz.so`` (hand-written HIP for
gfx950, declared in ``include/helmz.h``); this package is its Python binding.
"""

from .binding import (  # noqa: F401
    BREAKDOWN,
    NONFINITE,
    NOT_CONVERGED,
    OK,
    PRECOND_JACOBI,
    PRECOND_NONE,
    NO_REORDER,
    REORDER,
    SYMMETRIC,
    VALIDATE,
    X0_ZERO,
    autotune_spmv,
    csr_cspmv,
    csr_level_order,
    csr_reorder_workspace_bytes,
    csr_zpermute,
    csr_zgrad_vals,
    csr_zspmv,
    csr_zspmv_rect,
    dznrm2,
    handle,
    workspace,
    zaxpy,
    mixed_workspace,
    zbicgstab_mixed_workspace_bytes,
    zbicgstab_solve,
    zbicgstab_solve_mixed,
    zbicgstab_adjoint,
    zbicgstab_adjoint_batched,
    zbicgstab_adjoint_batched_workspace_bytes,
    zbicgstab_batched_workspace_bytes,
    zbicgstab_solve_batched,
    zbicgstab_varbatch_workspace_bytes,
    zbicgstab_solve_varbatch,
    zbicgstab_adjoint_workspace_bytes,
    zbicgstab_workspace_bytes,
    zdotc,
)
from .autograd import (  # noqa: F401
    EntryMap,
    HelmholtzSolve,
    HelmholtzSolveBatched,
    SolveOptions,
    entry_map,
    helmholtz_solve,
    helmholtz_solve_batched,
)
from ._lib import HelmzError, lib_path, load  # noqa: F401
