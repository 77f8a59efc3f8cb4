"""Python binding of the helmz C-ABI: torch tensors in, the same calls out.

Each function checks dtypes/devices/contiguity, passes ``data_ptr()`` and the
current HIP stream to the library, and returns torch tensors.  No arithmetic
of the method happens here; every step runs in the library's kernels.
"""

from __future__ import annotations

import ctypes as C
from ctypes import byref as C_byref, c_int64 as C_int64
import threading

import torch

from ._lib import HelmzError, HzC128, HzInfo, load

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, 2, 3
ERR_WORKSPACE = -3
ERR_TOO_LARGE = -4
PRECOND_NONE, PRECOND_JACOBI, X0_ZERO, VALIDATE, SYMMETRIC = 0x0, 0x1, 0x4, 0x8, 0x10
REORDER, NO_REORDER, RELIABLE = 0x20, 0x40, 0x80
BD_NONE, BD_RHO, BD_RHAT_V, BD_TT, BD_OMEGA, BD_MR = 0, 1, 2, 3, 4, 5  # info["breakdown"]: what became 0 / singular

_handles: dict[int, int] = {}
_hlock = threading.Lock()


def handle(device: torch.device | int | None = None) -> int:
    """Per-device library handle, created on first use with that device current."""
    if device is None:
        idx = torch.cuda.current_device()
    else:
        d = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = d.index if d.index is not None else torch.cuda.current_device()
    with _hlock:
        h = _handles.get(idx)
        if h is None:
            if torch.cuda.is_current_stream_capturing():
                raise RuntimeError("the library handle is created (device memory, a synchronised set-up kernel) on first "
                                   "use: call paper_2112_06465_amd.handle() before capturing a graph")
            with torch.cuda.device(idx):
                hp = C.c_void_p()
                rc = load().hz_handle_create(C.byref(hp))
                if rc != 0:
                    raise HelmzError("hz_handle_create", rc)
                h = hp.value
                _handles[idx] = h
    return h


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _need(t: torch.Tensor, name: str, dtype, dev=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if dev is not None and t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check(fn: str, rc: int, ok=(0,)):
    if rc not in ok:
        raise HelmzError(fn, rc)
    return rc


def _csr(row_ptr, col_idx, vals, vdtype):
    dev = vals.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    _need(vals, "vals", vdtype, dev)
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    if n < 0 or vals.numel() != nnz:
        raise ValueError("inconsistent CSR sizes")
    return dev, n, nnz


def csr_zspmv(row_ptr, col_idx, vals, x, y=None):
    """y = A x, complex128 CSR (csr_zspmv)."""
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(x, "x", torch.complex128, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    if y is None:
        y = torch.empty(n, dtype=torch.complex128, device=dev)
    _need(y, "y", torch.complex128, dev)
    rc = load().csr_zspmv(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(), vals.data_ptr(),
                          x.data_ptr(), y.data_ptr())
    _check("csr_zspmv", rc)
    return y


def _tune_key(row_ptr, col_idx, n, nnz):
    """Shape of a matrix for the tuning cache: device, n, nnz, longest row, default HYB width."""
    mx, width = csr_row_stats(row_ptr)
    name = torch.cuda.get_device_properties(row_ptr.device).name
    return f"{name}|n={n}|nnz={nnz}|maxrow={mx}|hyb={width}"


def _read_cache(path):
    import json

    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _write_cache(path, d):
    import json
    import os

    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_spmv(row_ptr, col_idx, vals, x=None, details=False, cache=None):
    """Time the launch shapes on this matrix and keep the fastest for it (hz_autotune_spmv).

    Returns the solver kernels' lane count; with details=True a dict with
    that count ("lanes"), the standalone product's form ("form": "rows" or
    "tiles") and its lane count ("form_lanes").  With ``cache`` (a JSON file
    path; default: the HZ_TUNE_CACHE environment variable) a choice stored
    for a matrix of the same shape (device, n, nnz, longest row, default HYB
    width) is recorded with hz_autotune_set instead of timing, and a new
    choice is added to the file.
    """
    import os

    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    cache = cache if cache is not None else os.environ.get("HZ_TUNE_CACHE")
    key = None
    if cache:
        key = _tune_key(row_ptr, col_idx, n, nnz)
        hit = _read_cache(cache).get(key)
        if hit is not None:
            rc = load().hz_autotune_set(handle(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                        int(hit["lanes"]), 1 if hit["form"] == "tiles" else 0, int(hit["form_lanes"]))
            _check("hz_autotune_set", rc)
            out = {"lanes": int(hit["lanes"]), "form": hit["form"], "form_lanes": int(hit["form_lanes"]),
                   "cached": True}
            return out if details else out["lanes"]
    if x is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        x = torch.randn(n, dtype=torch.complex128, generator=g).to(dev)
    _need(x, "x", torch.complex128, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    y = torch.empty(n, dtype=torch.complex128, device=dev)
    L, F, FL = C.c_int(0), C.c_int(0), C.c_int(0)
    rc = load().hz_autotune_spmv(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                 vals.data_ptr(), x.data_ptr(), y.data_ptr(), C.byref(L), C.byref(F), C.byref(FL))
    _check("hz_autotune_spmv", rc)
    out = {"lanes": int(L.value), "form": ("rows", "tiles")[F.value], "form_lanes": int(FL.value), "cached": False}
    if key is not None:
        d = _read_cache(cache)
        d[key] = {k: out[k] for k in ("lanes", "form", "form_lanes")}
        _write_cache(cache, d)
    return out if details else out["lanes"]


def csr_cspmv(row_ptr, col_idx, vals, x, y=None):
    """y = A x, complex64 CSR (csr_cspmv)."""
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex64)
    _need(x, "x", torch.complex64, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    if y is None:
        y = torch.empty(n, dtype=torch.complex64, device=dev)
    _need(y, "y", torch.complex64, dev)
    rc = load().csr_cspmv(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(), vals.data_ptr(),
                          x.data_ptr(), y.data_ptr())
    _check("csr_cspmv", rc)
    return y


def zdotc(x, y, out=None):
    """sum conj(x_i) y_i as a 0-d complex128 GPU tensor (zdotc)."""
    dev = x.device
    _need(x, "x", torch.complex128, dev)
    _need(y, "y", torch.complex128, dev)
    if x.numel() != y.numel():
        raise ValueError("length mismatch")
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=dev)
    _need(out, "out", torch.complex128, dev)
    rc = load().zdotc(handle(dev), _stream(dev), x.numel(), x.data_ptr(), y.data_ptr(), out.data_ptr())
    _check("zdotc", rc)
    return out


def csr_zspmv_plan(row_ptr, col_idx, vals, plan=None):
    """Plan for products in the caller's numbering through a level-set renumbered copy (csr_zspmv_plan).

    Returns a dict (n, nnz, plan tensor) for ``csr_zspmv_planned``; rebuild it after vals change.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    need = int(load().csr_zspmv_plan_bytes(n, nnz))
    if plan is None:
        plan = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(plan, "plan", torch.uint8, dev)
    pp, pbytes = _aligned_ptr(plan, need)
    rc = load().csr_zspmv_plan(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                               vals.data_ptr(), pp, pbytes)
    _check("csr_zspmv_plan", rc)
    return {"n": n, "nnz": nnz, "plan": plan}


def csr_zspmv_planned(plan, x, y=None):
    """y = A x (caller's numbering) with a plan from csr_zspmv_plan (csr_zspmv_planned)."""
    p = plan["plan"]
    dev, n, nnz = p.device, plan["n"], plan["nnz"]
    _need(x, "x", torch.complex128, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", torch.complex128, dev)
    need = int(load().csr_zspmv_plan_bytes(n, nnz))
    pp, pbytes = _aligned_ptr(p, need)
    rc = load().csr_zspmv_planned(handle(dev), _stream(dev), n, nnz, pp, pbytes, x.data_ptr(), y.data_ptr())
    _check("csr_zspmv_planned", rc)
    return y


def stream_read(buf, out=None):
    """Sum of a device buffer's doubles by the bandwidth-calibration read (hz_stream_read)."""
    dev = buf.device
    if not buf.is_contiguous() or buf.numel() * buf.element_size() % 16:
        raise ValueError("buf must be contiguous with a size that is a multiple of 16 bytes")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=dev)
    _need(out, "out", torch.float64, dev)
    rc = load().hz_stream_read(handle(dev), _stream(dev), buf.data_ptr(), buf.numel() * buf.element_size(),
                               out.data_ptr())
    _check("hz_stream_read", rc)
    return out


def stream_copy(src, dst):
    """dst <- src bytewise by the bandwidth-calibration copy (hz_stream_copy)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous buffers of one size")
    rc = load().hz_stream_copy(handle(src.device), _stream(src.device), src.data_ptr(), dst.data_ptr(), nbytes)
    _check("hz_stream_copy", rc)
    return dst


def dznrm2(x, out=None):
    """||x||_2 as a 0-d float64 GPU tensor (dznrm2)."""
    dev = x.device
    _need(x, "x", torch.complex128, dev)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=dev)
    _need(out, "out", torch.float64, dev)
    rc = load().dznrm2(handle(dev), _stream(dev), x.numel(), x.data_ptr(), out.data_ptr())
    _check("dznrm2", rc)
    return out


def zaxpy(alpha: complex, x, y):
    """y <- alpha x + y in place (zaxpy); returns y."""
    dev = y.device
    _need(x, "x", torch.complex128, dev)
    _need(y, "y", torch.complex128, dev)
    if x.numel() != y.numel():
        raise ValueError("length mismatch")
    a = complex(alpha)
    rc = load().zaxpy(handle(dev), _stream(dev), y.numel(), HzC128(a.real, a.imag), x.data_ptr(), y.data_ptr())
    _check("zaxpy", rc)
    return y


def zbicgstab_workspace_bytes(n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_workspace_bytes(int(n), int(nnz), int(flags)))


def workspace(n: int, nnz: int, flags: int, device) -> torch.Tensor:
    """A caller-owned workspace tensor of the size the solver needs (256-byte aligned)."""
    nbytes = zbicgstab_workspace_bytes(n, nnz, flags)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return ws


def _aligned_ptr(ws: torch.Tensor, nbytes: int) -> tuple[int, int]:
    p = ws.data_ptr()
    off = (-p) % 256
    if ws.numel() - off < nbytes:
        raise ValueError("workspace too small")
    return p + off, ws.numel() - off


def zbicgstab_solve(row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000, flags=PRECOND_NONE | X0_ZERO, ws=None):
    """Solve A x = b by (preconditioned) BiCGStab on the GPU (zbicgstab_solve).

    Returns (x, info).  ``x`` is updated in place when given (its entry value
    is the initial guess unless X0_ZERO is in ``flags``).  Solver statuses
    other than OK are reported in info, not raised; argument and runtime
    errors raise HelmzError.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = zbicgstab_workspace_bytes(n, nnz, flags)
    if ws is None:
        ws = workspace(n, nnz, flags, dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    info = HzInfo()
    rc = load().zbicgstab_solve(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol), int(maxiter), int(flags), wp,
                                wbytes, C.byref(info))
    _check("zbicgstab_solve", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, info.as_dict()


def zbicgstabl_workspace_bytes(n: int, nnz: int, ell: int = 8, flags: int = 0) -> int:
    return int(load().zbicgstabl_workspace_bytes(n, nnz, ell, flags))


def zbicgstab_solve_noalloc(row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000,
                            flags=PRECOND_NONE | X0_ZERO, info=None):
    """Enqueue a BiCGStab solve that allocates nothing (zbicgstab_solve_noalloc).

    The library's static scratch is the workspace; x and info (a device
    hz_solve_info, decoded by ``read_info``) are the caller's.  Pass both to
    make the call itself free of allocations.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    if info is None:
        info = torch.empty(C.sizeof(HzInfo), dtype=torch.uint8, device=dev)
    _need(info, "info", torch.uint8, dev)
    if info.numel() < C.sizeof(HzInfo):
        raise ValueError("info is too small")
    rc = load().zbicgstab_solve_noalloc(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                        vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol), int(maxiter),
                                        int(flags), info.data_ptr())
    _check("zbicgstab_solve_noalloc", rc)
    return x, info


def zbicgstab_noalloc_max_bytes() -> int:
    return int(load().zbicgstab_noalloc_max_bytes())


def zbicgstabl_solve(row_ptr, col_idx, vals, b, x=None, ell=8, rtol=1e-8, maxcycles=2500,
                     flags=PRECOND_NONE | X0_ZERO, ws=None):
    """Solve A x = b by BiCGstab(ell) on the GPU (zbicgstabl_solve).  Returns (x, info).

    info["iterations"] counts cycles (each ell Bi-CG steps, 2 ell products).
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = zbicgstabl_workspace_bytes(n, nnz, ell, flags)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    info = HzInfo()
    rc = load().zbicgstabl_solve(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                 vals.data_ptr(), b.data_ptr(), x.data_ptr(), int(ell), float(rtol), int(maxcycles),
                                 int(flags), wp, wbytes, C.byref(info))
    _check("zbicgstabl_solve", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, info.as_dict()


def zbicgstab_solve_async(row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000,
                          flags=PRECOND_NONE | X0_ZERO, ws=None, info=None):
    """Enqueue a BiCGStab solve with no host wait (zbicgstab_solve_async).

    Returns (x, info) where info is a device tensor holding an hz_solve_info,
    filled when the stream reaches the end of the solve; ``read_info(info)``
    decodes it (and waits for it).
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = zbicgstab_workspace_bytes(n, nnz, flags | NO_REORDER)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    if info is None:
        info = torch.empty(C.sizeof(HzInfo), dtype=torch.uint8, device=dev)
    _need(info, "info", torch.uint8, dev)
    if info.numel() < C.sizeof(HzInfo):
        raise ValueError("info is too small")
    rc = load().zbicgstab_solve_async(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                      vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol), int(maxiter),
                                      int(flags), wp, wbytes, info.data_ptr())
    _check("zbicgstab_solve_async", rc)
    return x, info


def read_info(info) -> dict:
    """Decode a device hz_solve_info written by an asynchronous solve (copies it to the host)."""
    raw = bytes(info[: C.sizeof(HzInfo)].cpu().numpy().tobytes())
    return HzInfo.from_buffer_copy(raw).as_dict()


def ztfqmr_workspace_bytes(n: int, nnz: int, flags: int = 0) -> int:
    return int(load().ztfqmr_workspace_bytes(n, nnz, flags))


def ztfqmr_solve(row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000, flags=PRECOND_NONE | X0_ZERO,
                 ws=None):
    """Solve A x = b by TFQMR on the GPU (ztfqmr_solve).  Returns (x, info).

    The stopping test is the quasi-residual bound (info["relres_recursive"]);
    info["iterations"] counts full iterations (two products each).
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = ztfqmr_workspace_bytes(n, nnz, flags)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    info = HzInfo()
    rc = load().ztfqmr_solve(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                             vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol), int(maxiter), int(flags), wp,
                             wbytes, C.byref(info))
    _check("ztfqmr_solve", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, info.as_dict()


def zbicgstab_mixed_workspace_bytes(n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_mixed_workspace_bytes(int(n), int(nnz), int(flags)))


def mixed_workspace(n: int, nnz: int, flags: int, device) -> torch.Tensor:
    return torch.empty(zbicgstab_mixed_workspace_bytes(n, nnz, flags) + 256, dtype=torch.uint8, device=device)


def zbicgstab_solve_mixed(
    row_ptr,
    col_idx,
    vals,
    b,
    x=None,
    rtol=1e-10,
    inner_rtol=None,
    maxiter=20000,
    max_outer=None,
    flags=PRECOND_NONE | X0_ZERO,
    ws=None,
):
    """Complex64-inner BiCGStab with complex128 refinement (zbicgstab_solve_mixed).  Returns (x, info).

    Defaults: restarted refinement with inner_rtol 1e-4 and at most 50
    corrections; with RELIABLE in ``flags``, reliable updates every decade
    (inner_rtol 0.1) and at most 200 of them.
    """
    reliable = bool(flags & RELIABLE)
    if inner_rtol is None:
        inner_rtol = 0.1 if reliable else 1e-4
    if max_outer is None:
        max_outer = 200 if reliable else 50
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(b, "b", torch.complex128, dev)
    if b.numel() != n:
        raise ValueError("b has the wrong length")
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = zbicgstab_mixed_workspace_bytes(n, nnz, flags)
    if ws is None:
        ws = mixed_workspace(n, nnz, flags, dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    info = HzInfo()
    rc = load().zbicgstab_solve_mixed(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                      vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol), float(inner_rtol),
                                      int(maxiter), int(max_outer), int(flags), wp, wbytes, C.byref(info))
    _check("zbicgstab_solve_mixed", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, info.as_dict()


def csr_zspmv_rect(row_ptr, col_idx, vals, x, y=None):
    """y = A x for a rectangular complex128 CSR matrix with row_ptr.numel()-1 rows (csr_zspmv_rect)."""
    dev = vals.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    _need(vals, "vals", torch.complex128, dev)
    _need(x, "x", torch.complex128, dev)
    m, nnz = row_ptr.numel() - 1, col_idx.numel()
    if m < 0 or vals.numel() != nnz:
        raise ValueError("inconsistent CSR sizes")
    if y is None:
        y = torch.empty(m, dtype=torch.complex128, device=dev)
    _need(y, "y", torch.complex128, dev)
    rc = load().csr_zspmv_rect(handle(dev), _stream(dev), m, x.numel(), nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                               vals.data_ptr(), x.data_ptr(), y.data_ptr())
    _check("csr_zspmv_rect", rc)
    return y


def csr_zgrad_vals(row_ptr, col_idx, lam, x, out=None):
    """out[p] = -lam_i conj(x_j) on the pattern (csr_zgrad_vals)."""
    dev = lam.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    _need(lam, "lambda", torch.complex128, dev)
    _need(x, "x", torch.complex128, dev)
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if out is None:
        out = torch.empty(nnz, dtype=torch.complex128, device=dev)
    _need(out, "grad_vals", torch.complex128, dev)
    rc = load().csr_zgrad_vals(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                               lam.data_ptr(), x.data_ptr(), out.data_ptr())
    _check("csr_zgrad_vals", rc)
    return out


def zbicgstab_adjoint_workspace_bytes(n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_adjoint_workspace_bytes(int(n), int(nnz), int(flags)))


def zbicgstab_adjoint(row_ptr, col_idx, vals, x, grad_x, rtol=1e-10, maxiter=20000, flags=PRECOND_NONE,
                      want_grad_vals=True, ws=None):
    """Backward of x = A^{-1} b (zbicgstab_adjoint).  Returns (grad_b, grad_vals or None, info)."""
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(grad_x, "grad_x", torch.complex128, dev)
    if grad_x.numel() != n:
        raise ValueError("grad_x has the wrong length")
    grad_b = torch.empty(n, dtype=torch.complex128, device=dev)
    grad_vals = None
    if want_grad_vals:
        _need(x, "x", torch.complex128, dev)
        grad_vals = torch.empty(nnz, dtype=torch.complex128, device=dev)
    need = zbicgstab_adjoint_workspace_bytes(n, nnz, flags)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    info = HzInfo()
    rc = load().zbicgstab_adjoint(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                  vals.data_ptr(), x.data_ptr() if want_grad_vals else None, grad_x.data_ptr(),
                                  grad_b.data_ptr(), grad_vals.data_ptr() if want_grad_vals else None, float(rtol),
                                  int(maxiter), int(flags), wp, wbytes, C.byref(info))
    _check("zbicgstab_adjoint", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return grad_b, grad_vals, info.as_dict()


def _row_off_array(row_off):
    import numpy as np

    ro = np.ascontiguousarray(np.asarray(row_off, dtype=np.int32))
    if ro.ndim != 1 or ro.size < 2:
        raise ValueError("row_off must hold nsys + 1 offsets")
    return ro


def zbicgstab_varbatch_workspace_bytes(row_off, nnz: int, flags: int = 0) -> int:
    ro = _row_off_array(row_off)
    return int(load().zbicgstab_varbatch_workspace_bytes(ro.size - 1, ro.ctypes.data, int(nnz), int(flags)))


def zbicgstab_solve_varbatch(row_off, row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000,
                             flags=PRECOND_NONE | X0_ZERO, ws=None):
    """Solve the diagonal blocks of a block-diagonal system independently (zbicgstab_solve_varbatch).

    ``row_off`` (host, nsys + 1 offsets) delimits the systems.  Returns
    (x, [info per system]).
    """
    ro = _row_off_array(row_off)
    nsys = ro.size - 1
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    if int(ro[-1]) != n:
        raise ValueError("row_off[-1] must equal the number of rows")
    _need(b, "b", torch.complex128, dev)
    if x is None:
        x = torch.zeros(n, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    need = zbicgstab_varbatch_workspace_bytes(ro, nnz, flags)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    infos = (HzInfo * nsys)()
    rc = load().zbicgstab_solve_varbatch(handle(dev), _stream(dev), nsys, ro.ctypes.data, nnz, row_ptr.data_ptr(),
                                         col_idx.data_ptr(), vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol),
                                         int(maxiter), int(flags), wp, wbytes, C.cast(infos, C.c_void_p))
    _check("zbicgstab_solve_varbatch", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, [i.as_dict() for i in infos]


def zbicgstab_batched_workspace_bytes(nsys: int, n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_batched_workspace_bytes(int(nsys), int(n), int(nnz), int(flags)))


def zbicgstab_solve_batched(row_ptr, col_idx, vals, b, x=None, rtol=1e-8, maxiter=20000, flags=PRECOND_NONE | X0_ZERO,
                            ws=None):
    """Solve B systems on one sparsity pattern (zbicgstab_solve_batched).

    ``vals`` is (nnz, B) complex128 (column j = system j's values), ``b`` and
    ``x`` are (n, B).  Returns (x, [info per system]).
    """
    dev = vals.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    _need(vals, "vals", torch.complex128, dev)
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if vals.dim() != 2 or vals.shape[0] != nnz:
        raise ValueError("vals must be (nnz, B)")
    nsys = vals.shape[1]
    _need(b, "b", torch.complex128, dev)
    if tuple(b.shape) != (n, nsys):
        raise ValueError("b must be (n, B)")
    if x is None:
        x = torch.zeros(n, nsys, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    if tuple(x.shape) != (n, nsys):
        raise ValueError("x must be (n, B)")
    need = zbicgstab_batched_workspace_bytes(nsys, n, nnz, flags)
    if need == 0:
        raise ValueError("unsupported batch size")
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    infos = (HzInfo * nsys)()
    rc = load().zbicgstab_solve_batched(handle(dev), _stream(dev), nsys, n, nnz, row_ptr.data_ptr(),
                                        col_idx.data_ptr(), vals.data_ptr(), b.data_ptr(), x.data_ptr(), float(rtol),
                                        int(maxiter), int(flags), wp, wbytes, C.cast(infos, C.c_void_p))
    _check("zbicgstab_solve_batched", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, [i.as_dict() for i in infos]


def zbicgstab_sweep_workspace_bytes(nsys: int, n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_sweep_workspace_bytes(int(nsys), int(n), int(nnz), int(flags)))


def zbicgstab_solve_sweep(row_ptr, col_idx, K, M, Bmat, ks, b, x=None, rtol=1e-8, maxiter=20000,
                          flags=PRECOND_NONE | X0_ZERO, ws=None):
    """Frequency sweep A(k_j) = K - k_j^2 M + i k_j B on one pattern (zbicgstab_solve_sweep).

    ``K``, ``M``, ``Bmat`` are float64 GPU tensors of nnz entries, ``ks`` a
    sequence of nsys wavenumbers (host), ``b`` and ``x`` (n, nsys).  Returns
    (x, [info per system]).
    """
    import numpy as np

    dev = K.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    for t, name in ((K, "K"), (M, "M"), (Bmat, "Bmat")):
        _need(t, name, torch.float64, dev)
        if t.numel() != nnz:
            raise ValueError(f"{name} must hold nnz entries")
    kh = np.ascontiguousarray(np.asarray(ks, dtype=np.float64))
    nsys = kh.size
    _need(b, "b", torch.complex128, dev)
    if tuple(b.shape) != (n, nsys):
        raise ValueError("b must be (n, nsys)")
    if x is None:
        x = torch.zeros(n, nsys, dtype=torch.complex128, device=dev)
        flags |= X0_ZERO
    _need(x, "x", torch.complex128, dev)
    if tuple(x.shape) != (n, nsys):
        raise ValueError("x must be (n, nsys)")
    need = zbicgstab_sweep_workspace_bytes(nsys, n, nnz, flags)
    if need == 0:
        raise ValueError("unsupported number of wavenumbers")
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    infos = (HzInfo * nsys)()
    rc = load().zbicgstab_solve_sweep(handle(dev), _stream(dev), nsys, n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                      K.data_ptr(), M.data_ptr(), Bmat.data_ptr(), kh.ctypes.data, b.data_ptr(),
                                      x.data_ptr(), float(rtol), int(maxiter), int(flags), wp, wbytes,
                                      C.cast(infos, C.c_void_p))
    _check("zbicgstab_solve_sweep", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return x, [i.as_dict() for i in infos]


def zbicgstab_adjoint_batched_workspace_bytes(nsys: int, n: int, nnz: int, flags: int = 0) -> int:
    return int(load().zbicgstab_adjoint_batched_workspace_bytes(int(nsys), int(n), int(nnz), int(flags)))


def zbicgstab_adjoint_batched(row_ptr, col_idx, vals, x, grad_x, rtol=1e-10, maxiter=20000, flags=PRECOND_NONE,
                              want_grad_vals=True, ws=None):
    """Backward of a shared-pattern batch (zbicgstab_adjoint_batched).

    ``vals`` (nnz, B), ``x`` and ``grad_x`` (n, B).  Returns
    (grad_b (n, B), grad_vals (nnz, B) or None, [info per system]).
    """
    dev = vals.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    _need(vals, "vals", torch.complex128, dev)
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if vals.dim() != 2 or vals.shape[0] != nnz:
        raise ValueError("vals must be (nnz, B)")
    nsys = vals.shape[1]
    _need(grad_x, "grad_x", torch.complex128, dev)
    if tuple(grad_x.shape) != (n, nsys):
        raise ValueError("grad_x must be (n, B)")
    grad_b = torch.empty(n, nsys, dtype=torch.complex128, device=dev)
    grad_vals = None
    if want_grad_vals:
        _need(x, "x", torch.complex128, dev)
        if tuple(x.shape) != (n, nsys):
            raise ValueError("x must be (n, B)")
        grad_vals = torch.empty(nnz, nsys, dtype=torch.complex128, device=dev)
    need = zbicgstab_adjoint_batched_workspace_bytes(nsys, n, nnz, flags)
    if need == 0:
        raise ValueError("unsupported batch size")
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    wp, wbytes = _aligned_ptr(ws, need)
    infos = (HzInfo * nsys)()
    rc = load().zbicgstab_adjoint_batched(handle(dev), _stream(dev), nsys, n, nnz, row_ptr.data_ptr(),
                                          col_idx.data_ptr(), vals.data_ptr(), x.data_ptr() if want_grad_vals else None,
                                          grad_x.data_ptr(), grad_b.data_ptr(),
                                          grad_vals.data_ptr() if want_grad_vals else None, float(rtol), int(maxiter),
                                          int(flags), wp, wbytes, C.cast(infos, C.c_void_p))
    _check("zbicgstab_adjoint_batched", rc, ok=(OK, NOT_CONVERGED, BREAKDOWN, NONFINITE))
    return grad_b, grad_vals, [i.as_dict() for i in infos]


def csr_reorder_workspace_bytes(n: int, nnz: int) -> int:
    return int(load().csr_reorder_workspace_bytes(int(n), int(nnz)))


def _reorder_ws(n: int, nnz: int, dev, ws):
    need = csr_reorder_workspace_bytes(n, nnz)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    return _aligned_ptr(ws, need), ws


# ------------------------------------------------------------------ storage formats (ELL / HYB, SELL-C-sigma)


def _fmt_ws(n, dev, ws):
    need = int(load().csr_format_workspace_bytes(n))
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    _need(ws, "ws", torch.uint8, dev)
    return _aligned_ptr(ws, need), ws


def csr_row_stats(row_ptr, ws=None):
    """(longest row, default HYB width) of a CSR pattern (csr_row_stats)."""
    dev = row_ptr.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    n = row_ptr.numel() - 1
    (wp, wbytes), _ws = _fmt_ws(n, dev, ws)
    mx, K = C.c_int(), C.c_int()
    rc = load().csr_row_stats(handle(dev), _stream(dev), n, row_ptr.data_ptr(), wp, wbytes, C.byref(mx), C.byref(K))
    _check("csr_row_stats", rc)
    return mx.value, K.value


def csr_to_hyb(row_ptr, col_idx, vals, K=None, ws=None):
    """HYB (ELL of width K plus COO remainder) of a CSR matrix (csr_to_hyb).

    K=None takes the default width, K="ell" the longest row (plain ELL).
    Returns a dict with n, K, ell_col [K*n], ell_val [K*n], coo_row, coo_col, coo_val.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    mx, Kd = csr_row_stats(row_ptr, ws)
    K = Kd if K is None else (mx if K == "ell" else int(K))
    (wp, wbytes), _ws = _fmt_ws(n, dev, ws)
    ell_col = torch.empty(K * n, dtype=torch.int32, device=dev)
    ell_val = torch.empty(K * n, dtype=torch.complex128, device=dev)
    cnt = C.c_int()
    lib, h, st = load(), handle(dev), _stream(dev)
    args = (h, st, n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(), vals.data_ptr(), K, ell_col.data_ptr(),
            ell_val.data_ptr())
    rc = lib.csr_to_hyb(*args, 0, None, None, None, wp, wbytes, C.byref(cnt))
    _check("csr_to_hyb", rc, ok=(OK, ERR_WORKSPACE))
    m = cnt.value
    coo_row = torch.empty(m, dtype=torch.int32, device=dev)
    coo_col = torch.empty(m, dtype=torch.int32, device=dev)
    coo_val = torch.empty(m, dtype=torch.complex128, device=dev)
    if rc != OK:
        rc = lib.csr_to_hyb(*args, m, coo_row.data_ptr(), coo_col.data_ptr(), coo_val.data_ptr(), wp, wbytes,
                            C.byref(cnt))
        _check("csr_to_hyb", rc)
    return {"n": n, "K": K, "ell_col": ell_col, "ell_val": ell_val, "coo_row": coo_row, "coo_col": coo_col,
            "coo_val": coo_val}


def hyb_zspmv(hyb, x, y=None):
    """y = A x with A in HYB storage (hyb_zspmv)."""
    dev, n = x.device, hyb["n"]
    _need(x, "x", torch.complex128, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", torch.complex128, dev)
    m = hyb["coo_row"].numel()
    rc = load().hyb_zspmv(handle(dev), _stream(dev), n, hyb["K"], hyb["ell_col"].data_ptr(),
                          hyb["ell_val"].data_ptr(), m, hyb["coo_row"].data_ptr(), hyb["coo_col"].data_ptr(),
                          hyb["coo_val"].data_ptr(), x.data_ptr(), y.data_ptr())
    _check("hyb_zspmv", rc)
    return y


def csr_to_sell(row_ptr, col_idx, vals, C=64, sigma=None, t=1, ws=None):
    """SELL-C-sigma with t lanes per row (csr_sell_analyze + csr_to_sell).

    sigma=None sorts within windows of 32 chunks (32 C rows).  Returns a dict
    with n, C, t, sigma, perm [n], chunk_ptr [ceil(n/C)+1] (int64), col, val.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    sigma = 32 * C if sigma is None else int(sigma)
    (wp, wbytes), _ws = _fmt_ws(n, dev, ws)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n]
    chunk_ptr = torch.empty((n + C - 1) // C + 1 if C >= 1 else 1, dtype=torch.int64, device=dev)
    slots = C_int64()
    lib, h, st = load(), handle(dev), _stream(dev)
    rc = lib.csr_sell_analyze(h, st, n, row_ptr.data_ptr(), C, sigma, t, perm.data_ptr(), chunk_ptr.data_ptr(), wp,
                              wbytes, C_byref(slots))
    _check("csr_sell_analyze", rc)
    col = torch.empty(slots.value, dtype=torch.int32, device=dev)
    val = torch.empty(slots.value, dtype=torch.complex128, device=dev)
    rc = lib.csr_to_sell(h, st, n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(), vals.data_ptr(), C, t,
                         perm.data_ptr(), chunk_ptr.data_ptr(), slots.value, col.data_ptr(), val.data_ptr())
    _check("csr_to_sell", rc)
    return {"n": n, "C": C, "t": t, "sigma": sigma, "perm": perm, "chunk_ptr": chunk_ptr, "col": col, "val": val}


def sell_zspmv(sell, x, y=None):
    """y = A x with A in SELL-C-sigma storage (sell_zspmv)."""
    dev, n = x.device, sell["n"]
    _need(x, "x", torch.complex128, dev)
    if x.numel() != n:
        raise ValueError("x has the wrong length")
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", torch.complex128, dev)
    rc = load().sell_zspmv(handle(dev), _stream(dev), n, sell["C"], sell["t"], sell["perm"].data_ptr(),
                           sell["chunk_ptr"].data_ptr(), sell["col"].data_ptr(), sell["val"].data_ptr(),
                           x.data_ptr(), y.data_ptr())
    _check("sell_zspmv", rc)
    return y


def csr_level_order(row_ptr, col_idx, ws=None):
    """Level-set (breadth-first) ordering of a CSR pattern (csr_level_order).

    Returns (perm, inv, level) as int32 GPU tensors: perm[k] = the caller's
    index of new row k, inv its inverse, level the breadth-first level of
    each caller index (-1 if unreached).
    """
    dev = row_ptr.device
    _need(row_ptr, "row_ptr", torch.int32, dev)
    _need(col_idx, "col_idx", torch.int32, dev)
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if n < 0:
        raise ValueError("row_ptr must hold n + 1 entries")
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    inv = torch.empty(n, dtype=torch.int32, device=dev)
    level = torch.empty(n, dtype=torch.int32, device=dev)
    (wp, wbytes), _ws = _reorder_ws(n, nnz, dev, ws)
    rc = load().csr_level_order(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                perm.data_ptr(), inv.data_ptr(), level.data_ptr(), wp, wbytes)
    _check("csr_level_order", rc)
    return perm, inv, level


def csr_zpermute(row_ptr, col_idx, vals, perm, inv, ws=None):
    """P A P^T in CSR for perm (new -> old) with inverse inv (csr_zpermute).

    Returns (row_ptr, col_idx, vals) of the renumbered matrix.
    """
    dev, n, nnz = _csr(row_ptr, col_idx, vals, torch.complex128)
    _need(perm, "perm", torch.int32, dev)
    _need(inv, "inv", torch.int32, dev)
    if perm.numel() != n or inv.numel() != n:
        raise ValueError("perm and inv must hold n entries")
    rp2 = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ci2 = torch.empty(nnz, dtype=torch.int32, device=dev)
    v2 = torch.empty(nnz, dtype=torch.complex128, device=dev)
    (wp, wbytes), _ws = _reorder_ws(n, nnz, dev, ws)
    rc = load().csr_zpermute(handle(dev), _stream(dev), n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                             vals.data_ptr(), perm.data_ptr(), inv.data_ptr(), rp2.data_ptr(), ci2.data_ptr(),
                             v2.data_ptr(), wp, wbytes)
    _check("csr_zpermute", rc)
    return rp2, ci2, v2
