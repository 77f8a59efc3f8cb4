"""The C-ABI library loads and exports every entry point its header declares (CPU only, no compute)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmz.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "defined")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("csr_zspmv", "zdotc", "dznrm2", "zaxpy", "zbicgstab_solve", "zbicgstab_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2112_06465_amd import build as B

    if B.stale():
        B.build()
    lib = ctypes.CDLL(B.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2112_06465_amd._lib import SIGNATURES

    assert set(declared_functions()) <= set(SIGNATURES)


def test_strerror_and_workspace_without_gpu():
    from paper_2112_06465_amd import _lib

    L = _lib.load()
    for code in (0, 1, 2, 3, -1, -2, -3, 99):
        assert isinstance(_lib.strerror(code), str) and _lib.strerror(code)
    # workspace size grows with n and with the Jacobi values copy
    a = L.zbicgstab_workspace_bytes(1000, 7000, 0)
    b = L.zbicgstab_workspace_bytes(1000, 7000, 1)
    assert b >= a + 16 * 7000 and a >= 6 * 16 * 1000
    assert L.zbicgstab_workspace_bytes(-1, 0, 0) == 0
