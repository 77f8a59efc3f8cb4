"""ctypes loader for ``libhelmz.so``.

The library is required: there is no CPU fallback.  If it is missing it is
built once from the in-tree sources with hipcc; if that fails, import-time
use raises.
"""

from __future__ import annotations

import ctypes as C
import os
import threading

from . import build as _build

_lock = threading.Lock()
_lib = None


class HzInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("iterations", C.c_int),
        ("outer_steps", C.c_int),
        ("renumbered", C.c_int),
        ("relres_recursive", C.c_double),
        ("relres_true", C.c_double),
        ("breakdown", C.c_int),
        ("reserved", C.c_int),
    ]

    def as_dict(self) -> dict:
        return {
            "status": self.status,
            "iterations": self.iterations,
            "outer_steps": self.outer_steps,
            "renumbered": self.renumbered,
            "relres_recursive": self.relres_recursive,
            "relres_true": self.relres_true,
            "breakdown": self.breakdown,
        }


class HzC128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


# name -> (restype, argtypes); mirrors include/helmz.h
P, I, D, SZ = C.c_void_p, C.c_int, C.c_double, C.c_size_t
SIGNATURES = {
    "hz_handle_create": (I, [C.POINTER(C.c_void_p)]),
    "hz_handle_destroy": (I, [P]),
    "hz_strerror": (C.c_char_p, [I]),
    "csr_zspmv": (I, [P, P, I, I, P, P, P, P, P]),
    "csr_cspmv": (I, [P, P, I, I, P, P, P, P, P]),
    "zdotc": (I, [P, P, I, P, P, P]),
    "dznrm2": (I, [P, P, I, P, P]),
    "zaxpy": (I, [P, P, I, HzC128, P, P]),
    "zbicgstab_workspace_bytes": (SZ, [I, I, I]),
    "zbicgstab_solve": (I, [P, P, I, I, P, P, P, P, P, D, I, I, P, SZ, C.POINTER(HzInfo)]),
    "zbicgstabl_workspace_bytes": (SZ, [I, I, I, I]),
    "zbicgstabl_solve": (I, [P, P, I, I, P, P, P, P, P, I, D, I, I, P, SZ, C.POINTER(HzInfo)]),
    "ztfqmr_workspace_bytes": (SZ, [I, I, I]),
    "zbicgstab_solve_async": (I, [P, P, I, I, P, P, P, P, P, D, I, I, P, SZ, P]),
    "ztfqmr_solve": (I, [P, P, I, I, P, P, P, P, P, D, I, I, P, SZ, C.POINTER(HzInfo)]),
    "csr_format_workspace_bytes": (SZ, [I]),
    "csr_row_stats": (I, [P, P, I, P, P, SZ, C.POINTER(I), C.POINTER(I)]),
    "csr_to_hyb": (I, [P, P, I, I, P, P, P, I, P, P, I, P, P, P, P, SZ, C.POINTER(I)]),
    "hyb_zspmv": (I, [P, P, I, I, P, P, I, P, P, P, P, P]),
    "csr_sell_analyze": (I, [P, P, I, P, I, I, I, P, P, P, SZ, C.POINTER(C.c_int64)]),
    "csr_to_sell": (I, [P, P, I, I, P, P, P, I, I, P, P, C.c_int64, P, P]),
    "sell_zspmv": (I, [P, P, I, I, I, P, P, P, P, P, P]),
    "zbicgstab_mixed_workspace_bytes": (SZ, [I, I, I]),
    "zbicgstab_varbatch_workspace_bytes": (SZ, [I, P, I, I]),
    "zbicgstab_solve_varbatch": (I, [P, P, I, P, I, P, P, P, P, P, D, I, I, P, SZ, P]),
    "zbicgstab_batched_workspace_bytes": (SZ, [I, I, I, I]),
    "zbicgstab_solve_batched": (I, [P, P, I, I, I, P, P, P, P, P, D, I, I, P, SZ, P]),
    "zbicgstab_sweep_workspace_bytes": (SZ, [I, I, I, I]),
    "zbicgstab_solve_sweep": (I, [P, P, I, I, I, P, P, P, P, P, P, P, P, D, I, I, P, SZ, P]),
    "csr_zspmv_rect": (I, [P, P, I, I, I, P, P, P, P, P]),
    "csr_zgrad_vals": (I, [P, P, I, I, P, P, P, P, P]),
    "zbicgstab_adjoint_workspace_bytes": (SZ, [I, I, I]),
    "zbicgstab_adjoint": (I, [P, P, I, I, P, P, P, P, P, P, P, D, I, I, P, SZ, C.POINTER(HzInfo)]),
    "zbicgstab_solve_mixed": (I, [P, P, I, I, P, P, P, P, P, D, D, I, I, I, P, SZ, C.POINTER(HzInfo)]),
    "csr_reorder_workspace_bytes": (SZ, [I, I]),
    "hz_autotune_spmv": (I, [P, P, I, I, P, P, P, P, P, C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
    "hz_autotune_set": (I, [P, I, I, P, P, I, I, I]),
    "zbicgstab_adjoint_batched_workspace_bytes": (SZ, [I, I, I, I]),
    "zbicgstab_adjoint_batched": (I, [P, P, I, I, I, P, P, P, P, P, P, P, D, I, I, P, SZ, P]),
    "csr_level_order": (I, [P, P, I, I, P, P, P, P, P, P, SZ]),
    "csr_zpermute": (I, [P, P, I, I, P, P, P, P, P, P, P, P, P, SZ]),
    "hz_stream_read": (I, [P, P, P, SZ, P]),
    "zbicgstab_noalloc_max_bytes": (SZ, []),
    "csr_zspmv_plan_bytes": (SZ, [I, I]),
    "csr_zspmv_plan": (I, [P, P, I, I, P, P, P, P, SZ]),
    "csr_zspmv_planned": (I, [P, P, I, I, P, SZ, P, P]),
    "zbicgstab_solve_noalloc": (I, [P, P, I, I, P, P, P, P, P, D, I, I, P]),
    "hz_stream_copy": (I, [P, P, P, P, SZ]),
}


def lib_path() -> str:
    return _build.LIB


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB):
                _build.build()
            L = C.CDLL(_build.LIB)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def strerror(code: int) -> str:
    return load().hz_strerror(int(code)).decode()


class HelmzError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {code} ({strerror(code)})")
        self.code = code
