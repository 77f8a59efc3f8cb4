#!/usr/bin/env python3
"""Benchmark of the Helmholtz BiCGStab hot path on one MI355X.

Headline workload: the cabin (P1 Kuhn-tet FEM on a 2.0 x 1.2 x 1.1 box with two
seat cutouts, h = 0.012, k = 40, node numbering randomly permuted:
n = 1,244,530, nnz = 18,213,332; 409 MB of algorithmic SpMV bytes, more than the
256 MB Infinity Cache, so the product streams from HBM).

One step = the whole hot path on the cabin:
  1. R standalone complex128 SpMVs (csr_zspmv) of the matrix after the
     library's level-set renumbering (csr_level_order + csr_zpermute, done once
     at set-up like the autotuning), alternating between 2 replicas so every
     launch reads cold data, bracketed by one pair of HIP events on the launch
     stream;
  2. one zdotc and one zaxpy on the n-vectors;
  3. one Jacobi-BiCGStab solve of A x = b to ||r||/||b|| <= 1e-10 in the
     caller's (random) numbering; the solve renumbers inside the call.

``value`` = zSpMV GB/s: algorithmic bytes of one product (20 nnz + 36 n + 4:
vals 16 and col_idx 4 per entry, row_ptr 4, x 16 and y 16 per row) / the
HIP-event average launch time over the timed steps.  ``roofline`` is that kernel
against the 8 TB/s HBM peak, beside a measured ceiling (hz_stream_read over
2 GiB).  ``step`` gives the whole step's algorithmic bytes / wall time.
``cpu_baseline`` times the oracle (sequential and its OpenMP build on all host
cores) on the same product and a bounded number of BiCGStab iterations.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --calib-copy          (hand-written 512 MiB copy, for counter scaling)
       python bench.py --profile WHAT        (one kernel family only, for rocprofv3)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
CABIN_REPLICAS = 2  # 2 x 409 MB > the 256 MB Infinity Cache
CYL_REPLICAS = 6  # 6 x 68.5 MB > the 256 MB Infinity Cache
CABIN_FORM = "tiles"  # the autotuner's pick on the renumbered cabin (block tiles)


def spmv_kernel_name(form, L=8, n=None):
    """Name of the standalone zSpMV kernel for a form ("rows" / "tiles") and lane count (tiles: one block per
    64-row tile below 4,096 tiles, else 1,024 blocks looping over them)."""
    if form == "tiles":
        return "hz::k_spmv_tile1<double>" if n is not None and -(-n // 64) < 4096 else "hz::k_spmv_tile<double>"
    U = 4 if L <= 4 else (2 if L == 8 else 1)
    return f"hz::k_spmv_pipe<double, {L}, {U}>"


def rule_lanes(n, nnz):
    L = 2
    while L < 64 and 2 * L < nnz / n:
        L *= 2
    return L


def spmv_bytes(n, nnz):
    return 20 * nnz + 36 * n + 4


def iter_bytes(n, nnz, fused):
    """Algorithmic bytes of one BiCGStab iteration (Jacobi folded): fused 3 launches / gather-light 5."""
    return 40 * nnz + (280 if fused else 344) * n


def solve_bytes(n, nnz, iterations, fused=False):
    return iterations * iter_bytes(n, nnz, fused) + 76 * nnz + 168 * n


def kernel_source_hash() -> str:
    """Hash of the device source of the standalone SpMV kernels (hz_spmv.hpp and hz_kernels.hpp)."""
    h = hashlib.sha256()
    for f in ("hz_spmv.hpp", "hz_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2112_06465_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(summary, kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary, if its kernel hash is current."""
    try:
        txt = open(os.path.join(PROFILES, summary)).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel source hash:\s*`?([0-9a-f]{16})", txt)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    m_bytes = re.search(r"HBM bytes per launch \(scaled\), `" + re.escape(kernel) + r"`:\s*([0-9.eE+]+)", txt)
    return float(m_bytes.group(1)) if m_bytes else None


def host_relres(A, x, b):
    """||b - A x|| / ||b|| on the host with scipy's sparse product (a check, not the oracle)."""
    import scipy.sparse as sp

    M = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return float(np.linalg.norm(b - M @ x) / np.linalg.norm(b))


def cached(cache_dir, name, make):
    """CSR + vectors of a workload, generated once per cache directory (profiling runs reuse them)."""
    import workloads as W

    if not cache_dir:
        return make()
    path = os.path.join(cache_dir, name + ".npz")
    if os.path.exists(path):
        z = np.load(path)
        return W.CSR(z["rp"], z["ci"], z["v"]), z["b"], {}
    A, b, info = make()
    os.makedirs(cache_dir, exist_ok=True)
    np.savez(path, rp=A.row_ptr, ci=A.col_idx, v=A.vals, b=b)
    return A, b, info


# ---------------------------------------------------------------- timing helpers


class ColdLoop:
    """R launches of one product cycling through replicas, one HIP event pair on the launch stream.

    One launch is enqueued ahead of the start event so that the GPU is busy when the timed region opens and
    the host's first call is not counted as idle time.
    """

    def __init__(self, torch, launch, replicas, reps):
        self.torch, self.launch, self.replicas, self.reps = torch, launch, replicas, reps
        self.ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def enqueue(self):
        self.launch(self.replicas[-1])
        self.ev[0].record()
        for r in range(self.reps):
            self.launch(self.replicas[r % len(self.replicas)])
        self.ev[1].record()

    def us(self):
        self.torch.cuda.synchronize()
        return self.ev[0].elapsed_time(self.ev[1]) * 1e3 / self.reps


def rate(nbytes, us):
    gbs = nbytes / (us * 1e-6) / 1e9
    return {"us": round(us, 3), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


class PinnedForm:
    """Pin the standalone product's form (and lane count) for the launches inside the block."""

    def __init__(self, form, lanes=None):
        self.form, self.lanes = form, lanes

    def __enter__(self):
        os.environ["HZ_SPMV_FORM"] = self.form
        if self.lanes:
            os.environ["HZ_SPMV_LANES"] = str(self.lanes)

    def __exit__(self, *a):
        os.environ.pop("HZ_SPMV_FORM", None)
        os.environ.pop("HZ_SPMV_LANES", None)


# ---------------------------------------------------------------- set-up of the workloads


class Cabin:
    """The cabin on the device: caller's (random) numbering and the level-set renumbered copy."""

    def __init__(self, hz, torch, dev, cache_dir=None):
        import workloads as W

        self.A, self.b_np, _ = cached(cache_dir, "cabin", W.config_cabin)
        A = self.A
        self.n, self.nnz = A.n, A.nnz
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        self.rp, self.ci, self.vals, self.b = up(A.row_ptr), up(A.col_idx), up(A.vals), up(self.b_np)
        rng = np.random.default_rng(1)
        self.x = up(rng.standard_normal(self.n) + 1j * rng.standard_normal(self.n))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.perm, self.inv, level = hz.csr_level_order(self.rp, self.ci)
        self.rp2, self.ci2, self.v2 = hz.csr_zpermute(self.rp, self.ci, self.vals, self.perm, self.inv)
        torch.cuda.synchronize()
        self.analysis_ms = (time.perf_counter() - t0) * 1e3
        self.levels = int(level.max().item()) + 1
        self.xp = self.x[self.perm.long()].contiguous()

    def replicas(self, torch, level=True):
        """CABIN_REPLICAS copies (matrix, x, y) in the level-set or the caller's numbering."""
        src = (self.rp2, self.ci2, self.v2, self.xp) if level else (self.rp, self.ci, self.vals, self.x)
        reps = [tuple(src) + (torch.empty_like(self.x),)]
        for _ in range(CABIN_REPLICAS - 1):
            reps.append(tuple(a.clone() for a in src) + (torch.empty_like(self.x),))
        return reps


# ---------------------------------------------------------------- sections


def stream_ceiling(hz, torch, dev, reps=10):
    """Hand-written read-only stream (hz_stream_read) and copy (hz_stream_copy): the ceiling on this part."""
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    out = torch.empty((), dtype=torch.float64, device=dev)
    res = {}
    for label, nbytes in (("read_2GiB", 2 << 30), ("read_409MB", 409_322_336)):
        bufs = [torch.ones(nbytes // 8, dtype=torch.float64, device=dev) for _ in range(2 if nbytes < 1 << 30 else 1)]
        hz.stream_read(bufs[-1], out=out)
        ev[0].record()
        for r in range(reps):
            hz.stream_read(bufs[r % len(bufs)], out=out)
        ev[1].record()
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        ok = out.item() == float(nbytes // 8)
        res[label] = dict(rate(nbytes, us), bytes=nbytes, sum_checked=ok)
        del bufs
    src = torch.ones((1 << 30) // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    hz.stream_copy(src, dst)
    ev[0].record()
    for _ in range(reps):
        hz.stream_copy(src, dst)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    res["copy_1GiB"] = dict(rate(2 << 30, us), bytes_moved=2 << 30, checked=bool(torch.equal(src, dst)))
    del src, dst
    torch.cuda.empty_cache()
    return res


def spmv_cabin(hz, torch, dev, cab, reps=20):
    """Cold zSpMV on the cabin: caller's numbering, level sets (rule rows, tuned, tiles) and ELL."""
    n, nnz = cab.n, cab.nnz
    res = {"workload": f"cabin (n={n}, nnz={nnz}), algorithmic bytes {spmv_bytes(n, nnz)}, "
                       f"{CABIN_REPLICAS} replicas, {reps} cold launches",
           "analysis_ms": round(cab.analysis_ms, 3), "levels": cab.levels}
    L = rule_lanes(n, nnz)
    launch = lambda r: hz.csr_zspmv(*r)  # noqa: E731
    for label, level, form in (("given_numbering", False, "rows"), ("given_numbering_tiles", False, "tiles"),
                               ("level_sets_rows", True, "rows"), ("level_sets_tiles", True, "tiles")):
        reps_ = cab.replicas(torch, level)
        with PinnedForm(form, L if form == "rows" else None):
            loop = ColdLoop(torch, launch, reps_, reps)
            loop.enqueue()
            res[label] = dict(rate(spmv_bytes(n, nnz), loop.us()), kernel=spmv_kernel_name(form, L))
        del reps_
    # the caller's numbering through a plan (level-set renumbered copy, x gathered, y scattered back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [hz.csr_zspmv_plan(cab.rp, cab.ci, cab.vals)]
    torch.cuda.synchronize()
    res["plan_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    plans.append(hz.csr_zspmv_plan(cab.rp, cab.ci, cab.vals.clone()))
    ys = [torch.empty_like(cab.x) for _ in plans]
    loop = ColdLoop(torch, lambda py: hz.csr_zspmv_planned(py[0], cab.x, py[1]), list(zip(plans, ys)), reps)
    loop.enqueue()
    res["given_numbering_planned"] = dict(rate(spmv_bytes(n, nnz), loop.us()),
                                          kernels="hz::k_gather_perm<double> + hz::k_spmv_tile<double>")
    del plans, ys
    torch.cuda.empty_cache()
    tune = hz.autotune_spmv(cab.rp2, cab.ci2, cab.v2, cab.xp, details=True)
    res["autotuned_form"] = {"form": tune["form"], "lanes": tune["form_lanes"]}
    ell = [hz.csr_to_hyb(cab.rp2, cab.ci2, cab.v2, K="ell")]
    ell.append({k: (v.clone() if hasattr(v, "clone") else v) for k, v in ell[0].items()})
    ys = [torch.empty_like(cab.x) for _ in ell]
    loop = ColdLoop(torch, lambda e: hz.hyb_zspmv(e[0], cab.xp, e[1]), list(zip(ell, ys)), reps)
    loop.enqueue()
    res["level_sets_ell"] = dict(rate(spmv_bytes(n, nnz), loop.us()), K=ell[0]["K"])
    del ell, ys
    torch.cuda.empty_cache()
    return res


def spmv_cylinder(hz, torch, dev, reps=30):
    """Cold zSpMV of the cylinder (68.5 MB): 6 replicas; CSR rule rows, CSR block tiles, ELL and SELL-64-1."""
    import workloads as W

    A, _, _ = W.config_cylinder()
    n, nnz = A.n, A.nnz
    rng = np.random.default_rng(3)
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    x = up(rng.standard_normal(n) + 1j * rng.standard_normal(n))
    rp, ci, vals = up(A.row_ptr), up(A.col_idx), up(A.vals)
    L = rule_lanes(n, nnz)
    res = {"workload": f"cylinder (n={n}, nnz={nnz}), {CYL_REPLICAS} replicas, {reps} cold launches",
           "algorithmic_bytes": spmv_bytes(n, nnz)}
    reps_ = [(rp, ci, vals, x, torch.empty_like(x))] + [
        (rp.clone(), ci.clone(), vals.clone(), x.clone(), torch.empty_like(x)) for _ in range(CYL_REPLICAS - 1)]
    for label, form, lanes in (("csr_rows", "rows", L), ("csr_tiles", "tiles", None)):
        with PinnedForm(form, lanes):
            loop = ColdLoop(torch, lambda r: hz.csr_zspmv(*r), reps_, reps)
            loop.enqueue()
            res[label] = dict(rate(spmv_bytes(n, nnz), loop.us()), kernel=spmv_kernel_name(form, L, n))
    del reps_
    for label, conv, prod, stored in (
        ("ell", lambda: hz.csr_to_hyb(rp.clone(), ci.clone(), vals.clone(), K="ell"), hz.hyb_zspmv,
         lambda f: 20 * f["K"] * n + 32 * n),
        ("sell_64_1", lambda: hz.csr_to_sell(rp.clone(), ci.clone(), vals.clone(), C=64, sigma=1, t=1),
         hz.sell_zspmv, lambda f: 20 * f["col"].numel() + 4 * n + 8 * f["chunk_ptr"].numel() + 32 * n),
    ):
        fs = [(conv(), x.clone(), torch.empty_like(x)) for _ in range(CYL_REPLICAS)]
        loop = ColdLoop(torch, lambda f: prod(*f), fs, reps)
        loop.enqueue()
        res[label] = dict(rate(spmv_bytes(n, nnz), loop.us()), stored_bytes=int(stored(fs[0][0])))
        del fs
    torch.cuda.empty_cache()
    return res


def time_solves(hz, torch, dev, name, A, b_np, rp, ci, vals, tol, runs, maxiter=50000, maxcycles=3125):
    """Wall time of each named solve to tol (one warm-up, then one timed run); x checked on the host."""
    n, nnz = A.n, A.nnz
    b = torch.from_numpy(b_np).to(dev)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    x = torch.zeros_like(b)
    res = {"workload": f"{name} (n={n}, nnz={nnz})", "tol": tol}
    wss = {}

    def ws(kind):
        if kind not in wss:
            nbytes = {"fp64": lambda: hz.zbicgstab_workspace_bytes(n, nnz, flags),
                      "mixed": lambda: hz.zbicgstab_mixed_workspace_bytes(n, nnz, flags),
                      "l8": lambda: hz.zbicgstabl_workspace_bytes(n, nnz, 8, flags),
                      "tfqmr": lambda: hz.ztfqmr_workspace_bytes(n, nnz, flags)}[kind]()
            wss[kind] = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        return wss[kind]

    table = {
        "fp64": lambda: hz.zbicgstab_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=maxiter, flags=flags,
                                           ws=ws("fp64")),
        "fp64_caller_order": lambda: hz.zbicgstab_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=maxiter,
                                                        flags=flags | hz.NO_REORDER, ws=ws("fp64")),
        "mixed": lambda: hz.zbicgstab_solve_mixed(rp, ci, vals, b, x=x, rtol=tol, inner_rtol=1e-4, maxiter=maxiter,
                                                  flags=flags, ws=ws("mixed")),
        "mixed_reliable": lambda: hz.zbicgstab_solve_mixed(rp, ci, vals, b, x=x, rtol=tol, maxiter=maxiter,
                                                           flags=flags | hz.RELIABLE, ws=ws("mixed")),
        # BiCGstab(8), the paper's second solver: iterations are cycles of 8 Bi-CG steps (16 products)
        "bicgstab_l8": lambda: hz.zbicgstabl_solve(rp, ci, vals, b, x=x, ell=8, rtol=tol, maxcycles=maxcycles,
                                                   flags=flags, ws=ws("l8")),
        # TFQMR, the paper's third solver: two products per iteration, stopped on the quasi-residual bound
        "tfqmr": lambda: hz.ztfqmr_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=maxiter, flags=flags,
                                         ws=ws("tfqmr")),
    }
    x64 = None
    for label in runs:
        fn = table[label]
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        xh = x.cpu().numpy()
        res[label] = {"ms": round(ms, 3), "iterations": info["iterations"], "outer_steps": info["outer_steps"],
                      "status": info["status"], "renumbered": info["renumbered"],
                      "relres_true_host": host_relres(A, xh, b_np)}
        if label == "fp64":
            x64 = xh.copy()
        elif x64 is not None:
            res[label]["rel_err_vs_fp64"] = float(np.linalg.norm(xh - x64) / np.linalg.norm(x64))
    if "fp64" in res:
        for label in runs:
            if label != "fp64" and res[label]["status"] == 0:
                res[label + "_speedup"] = round(res["fp64"]["ms"] / res[label]["ms"], 3)
    del wss
    torch.cuda.empty_cache()
    return res


def adjoint_cylinder(hz, torch, dev, tol=1e-10):
    """Backward pass on the full cylinder: L = sum_r |x_r - t_r|^2 over 1000 receivers, 50 sources.

    Timed: one adjoint solve A^H lambda = g (with grad_vals = -lambda_i conj(x_j) on the pattern) and the
    chain to the per-node impedance coefficients, grad_beta = Phi^H grad_vals (csr_zspmv_rect); the
    gradient w.r.t. the 50 source amplitudes is lambda at the source nodes.
    """
    import workloads as W

    A, cfg = W.config_adjoint()
    n, nnz = A.n, A.nnz
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rp, ci, vals = up(A.row_ptr), up(A.col_idx), up(A.vals)
    rec, t, src, amps = (up(cfg[k]) for k in ("receivers", "targets", "sources", "amps"))
    m = W.fem_impedance_map(A, cfg["parts"]["tris"], cfg["mesh"]["coords"], 20.0)
    phi_h = tuple(up(a) for a in m["phi_h"])
    b = torch.zeros(n, dtype=torch.complex128, device=dev).index_add(0, src.long(), amps)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    x, finfo = hz.zbicgstab_solve(rp, ci, vals, b, rtol=tol, flags=flags)
    g = torch.zeros_like(x)
    g[rec.long()] = 2 * (x[rec.long()] - t)
    aflags = hz.PRECOND_JACOBI | hz.SYMMETRIC
    wsa = torch.empty(hz.zbicgstab_adjoint_workspace_bytes(n, nnz, aflags) + 256, dtype=torch.uint8, device=dev)

    def backward():
        lam, gv, info = hz.zbicgstab_adjoint(rp, ci, vals, x, g, rtol=tol, flags=aflags, ws=wsa)
        gbeta = hz.csr_zspmv_rect(*phi_h, gv)
        return lam, gv, gbeta, info

    backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, gv, gbeta, info = backward()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    # lambda's residual on the host: A = A^T, so A^H lambda = conj(A conj(lambda))
    lam_h = lam.cpu().numpy()
    g_h = g.cpu().numpy()
    rr = host_relres(A, np.conj(lam_h), np.conj(g_h))
    it = info["iterations"]
    phi_nnz = int(phi_h[1].numel())
    nbytes = (solve_bytes(n, nnz, it) + (20 * nnz + 36 * n + 16 * nnz)
              + (20 * phi_nnz + 4 * (n + 1) + 16 * nnz + 16 * n))
    return {
        "workload": f"cylinder (n={n}, nnz={nnz}), 1000 receivers, 50 sources, per-node impedance via Phi "
                    f"({phi_nnz} entries), Jacobi, tol {tol:g}",
        "forward_iterations": finfo["iterations"],
        "backward_ms": round(ms, 3), "adjoint_iterations": it, "status": info["status"],
        "lambda_relres_host": rr,
        "algorithmic_bytes": nbytes, "algorithmic_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
        "byte_model": "adjoint solve (set-up + iterations x (40 nnz + 344 n)) + grad_vals (20 nnz + 36 n read, "
                      "16 nnz written) + Phi^H grad_vals (20 nnz(Phi) + 4 (n+1) + 16 nnz read, 16 n written)",
        "grad_amps_norm": float(lam[src.long()].abs().norm().item()),
        "grad_beta_norm": float(gbeta.abs().norm().item()),
    }


def blas1(hz, torch, dev, sizes=(100_000, 209_777, 1_000_000, 5_000_000, 15_000_000), reps=20):
    """Standalone zdotc / dznrm2 / zaxpy: per-call time of back-to-back calls and algorithmic GB/s."""
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    rng = np.random.default_rng(2)
    out = []
    for n in sizes:
        x = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(dev)
        y = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(dev)
        d = torch.empty((), dtype=torch.complex128, device=dev)
        nr = torch.empty((), dtype=torch.float64, device=dev)
        row = {"n": n}
        for name, fn, nbytes in (
            ("zdotc", lambda: hz.zdotc(x, y, out=d), 32 * n),
            ("dznrm2", lambda: hz.dznrm2(x, out=nr), 16 * n),
            ("zaxpy", lambda: hz.zaxpy(1e-9 - 1e-9j, x, y), 48 * n),
        ):
            for _ in range(3):
                fn()
            ev[0].record()
            for _ in range(reps):
                fn()
            ev[1].record()
            torch.cuda.synchronize()
            us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
            row[name] = {"us": round(us, 2), "GBs": round(nbytes / (us * 1e-6) / 1e9, 1)}
        if n == 209_777:
            row["in_graph"] = blas1_in_graph(hz, torch, x, y, d, nr, ev)
        out.append(row)
        del x, y
    return out


def blas1_in_graph(hz, torch, x, y, d, nr, ev, calls=20, replays=5):
    """Per-call time of zdotc / dznrm2 / zaxpy captured `calls` times in one CUDA graph, replayed `replays` times.

    These kernels record no memset nodes; every replay's dot and norm are checked against the eager result (the
    zaxpy graph is checked once, against the same calls run eagerly on a copy of y).
    """
    n = x.numel()
    res = {}
    ref_d = hz.zdotc(x, y, out=torch.empty_like(d)).item()
    ref_n = hz.dznrm2(x, out=torch.empty_like(nr)).item()
    for name, fn, nbytes, check in (
        ("zdotc", lambda: hz.zdotc(x, y, out=d), 32 * n, lambda: d.item() == ref_d),
        ("dznrm2", lambda: hz.dznrm2(x, out=nr), 16 * n, lambda: nr.item() == ref_n),
        ("zaxpy", lambda: hz.zaxpy(1e-9 - 1e-9j, x, y), 48 * n, None),
    ):
        y0 = y.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(calls):
                fn()
        torch.cuda.synchronize()
        ok = True
        if name == "zaxpy":
            y.copy_(y0)
            yy = y0.clone()
            for _ in range(calls):
                hz.zaxpy(1e-9 - 1e-9j, x, yy)
            g.replay()
            torch.cuda.synchronize()
            ok = bool(torch.equal(y, yy))
        ev[0].record()
        for _ in range(replays):
            g.replay()
        ev[1].record()
        torch.cuda.synchronize()
        if check is not None:
            for _ in range(replays):
                g.replay()
                torch.cuda.synchronize()
                ok = ok and check()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / (calls * replays)
        res[name] = {"us": round(us, 2), "GBs": round(nbytes / (us * 1e-6) / 1e9, 1), "replays_match_eager": ok}
        y.copy_(y0)
        del g
    return res


def batched_sweep(hz, torch, dev, B=64, tol=1e-10):
    """64 wavenumbers k ~ U[10, 40] on the cylinder pattern: one shared-pattern call vs 64 sequential solves."""
    import workloads as W

    A, vals, rhs, ks, sw = W.config_freq_sweep(B=B)
    n, nnz = A.n, A.nnz
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    V = torch.from_numpy(np.ascontiguousarray(vals.T)).to(dev)
    Bm = torch.from_numpy(np.ascontiguousarray(rhs.T)).to(dev)
    singles = [(torch.from_numpy(vals[j]).to(dev), torch.from_numpy(rhs[j]).to(dev)) for j in range(B)]
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    X = torch.zeros_like(Bm)
    wsb = torch.empty(hz.zbicgstab_batched_workspace_bytes(B, n, nnz, flags) + 256, dtype=torch.uint8, device=dev)
    ws = hz.workspace(n, nnz, flags, dev)
    xs = [torch.zeros_like(b) for _, b in singles]
    hz.zbicgstab_solve_batched(rp, ci, V, Bm, x=X, rtol=tol, maxiter=2, flags=flags, ws=wsb)
    hz.zbicgstab_solve(rp, ci, singles[0][0], singles[0][1], x=xs[0], rtol=tol, maxiter=2, flags=flags, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, binfo = hz.zbicgstab_solve_batched(rp, ci, V, Bm, x=X, rtol=tol, maxiter=50000, flags=flags, ws=wsb)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    sinfo = [hz.zbicgstab_solve(rp, ci, v, b, x=x, rtol=tol, maxiter=50000, flags=flags, ws=ws)[1]
             for (v, b), x in zip(singles, xs)]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    Kd, Md, Bd = (torch.from_numpy(sw[k]).to(dev) for k in ("K", "M", "B"))
    Xk = torch.zeros_like(Bm)
    wsk = torch.empty(hz.zbicgstab_sweep_workspace_bytes(B, n, nnz, flags) + 256, dtype=torch.uint8, device=dev)
    hz.zbicgstab_solve_sweep(rp, ci, Kd, Md, Bd, ks, Bm, x=Xk, rtol=tol, maxiter=2, flags=flags, ws=wsk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, kinfo = hz.zbicgstab_solve_sweep(rp, ci, Kd, Md, Bd, ks, Bm, x=Xk, rtol=tol, maxiter=50000, flags=flags,
                                        ws=wsk)
    torch.cuda.synchronize()
    t_k = time.perf_counter() - t0
    Xkh, Xh = Xk.cpu().numpy(), X.cpu().numpy()
    rr = lambda XX, j: host_relres(A.with_vals(vals[j]), XX[:, j], rhs[j])  # noqa: E731
    rr_k = max(rr(Xkh, j) for j in range(B))
    rr_b = max(rr(Xh, j) for j in range(B))
    rr_s = max(host_relres(A.with_vals(vals[j]), xs[j].cpu().numpy(), rhs[j]) for j in range(B))
    its = [i["iterations"] for i in binfo]
    return {
        "workload": f"{B} wavenumbers k~U[10,40] on the cylinder pattern (n={n}, nnz={nnz}), Jacobi, tol {tol:g}",
        "batched_ms": round(t_b * 1e3, 3), "sequential_ms": round(t_s * 1e3, 3), "speedup": round(t_s / t_b, 3),
        "from_K_M_B": {"ms": round(t_k * 1e3, 3), "speedup_vs_sequential": round(t_s / t_k, 3),
                       "iterations_min_max": [min(i["iterations"] for i in kinfo), max(i["iterations"] for i in kinfo)],
                       "all_ok": all(i["status"] == 0 for i in kinfo), "max_relres_true_host": rr_k},
        "iterations_min_max": [min(its), max(its)],
        "iterations_sequential_min_max": [min(i["iterations"] for i in sinfo), max(i["iterations"] for i in sinfo)],
        "all_ok": all(i["status"] == 0 for i in binfo) and all(i["status"] == 0 for i in sinfo),
        "max_relres_true_host": {"batched": rr_b, "sequential": rr_s},
        "batched_algorithmic_GBs": round((sum(its) * (32 * nnz + 304 * n) + max(its) * (8 * nnz + 8 * n)) / t_b / 1e9,
                                         1),
    }


def batched_cubes(hz, torch, dev, B=32, tols=(1e-8, 1e-10)):
    """32 independent 7-point cubes (N ~ U{16..64}, own k): one batched solve vs 32 sequential solves."""
    import workloads as W

    systems, info = W.config_cube_batch(B=B)
    row_off = np.zeros(B + 1, dtype=np.int64)
    rps, cis, vs, bs, nnz_off = [], [], [], [], 0
    for j, (A, b) in enumerate(systems):
        row_off[j + 1] = row_off[j] + A.n
        rps.append(A.row_ptr[:-1].astype(np.int64) + nnz_off)
        cis.append(A.col_idx.astype(np.int64) + row_off[j])
        vs.append(A.vals)
        bs.append(b)
        nnz_off += A.nnz
    rp = torch.from_numpy(np.concatenate(rps + [np.array([nnz_off])]).astype(np.int32)).to(dev)
    ci = torch.from_numpy(np.concatenate(cis).astype(np.int32)).to(dev)
    vv = torch.from_numpy(np.concatenate(vs)).to(dev)
    bb = torch.from_numpy(np.concatenate(bs)).to(dev)
    ro = row_off.astype(np.int32)
    xb = torch.zeros_like(bb)
    flags = hz.PRECOND_NONE | hz.X0_ZERO
    wsb = torch.empty(hz.zbicgstab_varbatch_workspace_bytes(ro, nnz_off, flags) + 256, dtype=torch.uint8, device=dev)
    singles = [tuple(torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.vals, b)) for A, b in systems]
    wss = hz.workspace(max(A.n for A, _ in systems), max(A.nnz for A, _ in systems), flags, dev)
    xs = [torch.zeros_like(s[3]) for s in singles]
    out = {"workload": f"{B} cubes N~U{{16..64}} (sum n={int(row_off[-1])}, nnz={nnz_off}), unpreconditioned"}
    for tol in tols:
        def run_batched():
            return hz.zbicgstab_solve_varbatch(ro, rp, ci, vv, bb, x=xb, rtol=tol, maxiter=50000, flags=flags,
                                               ws=wsb)

        def run_sequential():
            return [hz.zbicgstab_solve(*s, x=x, rtol=tol, maxiter=50000, flags=flags, ws=wss)
                    for s, x in zip(singles, xs)]

        res = {}
        for label, fn in (("batched", run_batched), ("sequential", run_sequential)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            res[label + "_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
            infos = r[1] if label == "batched" else [i for _, i in r]
            res[label + "_iterations_min_max"] = [min(i["iterations"] for i in infos),
                                                  max(i["iterations"] for i in infos)]
            res[label + "_all_ok"] = all(i["status"] == 0 for i in infos)
        xh = xb.cpu().numpy()
        res["max_relres_true_host"] = max(host_relres(A, xh[row_off[j]:row_off[j + 1]], b)
                                          for j, (A, b) in enumerate(systems))
        res["speedup"] = round(res["sequential_ms"] / res["batched_ms"], 3)
        out[f"tol_{tol:g}"] = res
    return out


def cpu_baseline(cab, min_seconds=4.0, iters=30):
    """The oracle on the host: the cabin product (sequential and the OpenMP build on all affinity cores) and a
    bounded number of Jacobi-BiCGStab iterations on the same matrix.  About 15-25 s in total."""
    import oracle as O
    import workloads as W

    A = W.CSR(cab.rp2.cpu().numpy(), cab.ci2.cpu().numpy(), cab.v2.cpu().numpy())
    x = cab.xp.cpu().numpy()
    n, nnz = A.n, A.nnz
    legs = {}
    for label, fn in (("single_thread", O.zspmv), ("all_cores", O.zspmv_omp)):
        fn(A, x)
        reps, t0 = 0, time.perf_counter()
        while True:
            fn(A, x)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                break
        legs[label] = {"GBs": round(spmv_bytes(n, nnz) * reps / dt / 1e9, 3), "ms_per_spmv": round(dt / reps * 1e3, 3),
                       "reps": reps, "cores": 1 if label == "single_thread" else O.omp_threads()}
    b = cab.b_np[cab.perm.cpu().numpy()]
    t0 = time.perf_counter()
    _, info = O.zbicgstab_omp(A, b, tol=1e-30, maxiter=iters, jacobi=True)
    dt = time.perf_counter() - t0
    legs["bicgstab_all_cores"] = {"iterations": info["iterations"], "ms_per_iteration": round(dt / iters * 1e3, 3),
                                  "GBs": round(iters * iter_bytes(n, nnz, False) / dt / 1e9, 3)}
    return {
        "value": legs["all_cores"]["GBs"],
        "unit": "GB/s",
        "cores": legs["all_cores"]["cores"],
        "kind": "oracle",
        "sample": f"the level-set renumbered cabin product (n={n}, nnz={nnz}), repeated for >= {min_seconds:g} s per "
                  f"leg, sequential and OpenMP builds of the plain C oracle (-O2, no FMA), on '{O.cpu_model()}' "
                  f"({O.affinity_cores()} affinity cores); plus {iters} Jacobi-BiCGStab iterations of the OpenMP "
                  f"build on the same matrix",
        "legs": legs,
    }


# ---------------------------------------------------------------- profiling and calibration modes


def calib_copy():
    """Five hand-written copies of 512 MiB (hz_stream_copy): counter scaling for rocprofv3."""
    import torch

    import paper_2112_06465_amd as hz

    nbytes = 512 * 2**20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        hz.stream_copy(src, dst)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes, "launches": 5, "kernel": "hz::k_stream_copy"}), flush=True)


def profile(what, steps, cache_dir):
    """Run one kernel family only (no autotuning, no other products), for rocprofv3 traces and counters."""
    import torch

    import paper_2112_06465_amd as hz

    dev = torch.device("cuda:0")
    if what.startswith("spmv-cabin"):
        cab = Cabin(hz, torch, dev, cache_dir)
        L = rule_lanes(cab.n, cab.nnz)
        if what == "spmv-cabin-planned":
            plans = [hz.csr_zspmv_plan(cab.rp, cab.ci, cab.vals), hz.csr_zspmv_plan(cab.rp, cab.ci, cab.vals.clone())]
            ys = [torch.empty_like(cab.x) for _ in plans]
            loop = ColdLoop(torch, lambda py: hz.csr_zspmv_planned(py[0], cab.x, py[1]), list(zip(plans, ys)), 30)
            form = None
        elif what == "spmv-cabin-ell":
            ell = [hz.csr_to_hyb(cab.rp2, cab.ci2, cab.v2, K="ell")]
            ell.append({k: (v.clone() if hasattr(v, "clone") else v) for k, v in ell[0].items()})
            ys = [torch.empty_like(cab.x) for _ in ell]
            loop = ColdLoop(torch, lambda e: hz.hyb_zspmv(e[0], cab.xp, e[1]), list(zip(ell, ys)), 30)
            form = None
        else:
            level = not what.startswith("spmv-cabin-given")
            form = {"spmv-cabin": CABIN_FORM, "spmv-cabin-rows": "rows", "spmv-cabin-given": "rows",
                    "spmv-cabin-given-tiles": "tiles"}[what]
            loop = ColdLoop(torch, lambda r: hz.csr_zspmv(*r), cab.replicas(torch, level), 30)
        for _ in range(steps):
            with PinnedForm(form or "rows", L if form == "rows" else None):
                loop.enqueue()
            print(what, "us per launch", round(loop.us(), 3), flush=True)
    elif what == "solve-cabin":
        cab = Cabin(hz, torch, dev, cache_dir)
        for _ in range(steps):
            t0 = time.perf_counter()
            _, info = hz.zbicgstab_solve(cab.rp, cab.ci, cab.vals, cab.b, rtol=1e-10, maxiter=50000,
                                         flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
            torch.cuda.synchronize()
            print(what, "ms", round(1e3 * (time.perf_counter() - t0), 2), info, flush=True)
    elif what in ("spmv-cylinder", "spmv-cylinder-rows"):
        import workloads as W

        A, _, _ = W.config_cylinder()
        n, nnz = A.n, A.nnz
        rng = np.random.default_rng(3)
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        x = up(rng.standard_normal(n) + 1j * rng.standard_normal(n))
        reps_ = [(up(A.row_ptr), up(A.col_idx), up(A.vals), x.clone(), torch.empty_like(x))
                 for _ in range(CYL_REPLICAS)]
        form = "tiles" if what == "spmv-cylinder" else "rows"
        loop = ColdLoop(torch, lambda r: hz.csr_zspmv(*r), reps_, 30)
        for _ in range(steps):
            with PinnedForm(form, rule_lanes(n, nnz) if form == "rows" else None):
                loop.enqueue()
            print(what, "us per launch", round(loop.us(), 3), flush=True)
    elif what == "solve-cabin-l8":
        cab = Cabin(hz, torch, dev, cache_dir)
        for _ in range(steps):
            t0 = time.perf_counter()
            _, info = hz.zbicgstabl_solve(cab.rp, cab.ci, cab.vals, cab.b, ell=8, rtol=1e-10, maxcycles=5000,
                                          flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
            torch.cuda.synchronize()
            print(what, "ms", round(1e3 * (time.perf_counter() - t0), 2), info, flush=True)
    elif what == "solve-cabin-mixed":
        cab = Cabin(hz, torch, dev, cache_dir)
        for _ in range(steps):
            for label, extra in (("restarted", 0), ("reliable", hz.RELIABLE)):
                t0 = time.perf_counter()
                _, info = hz.zbicgstab_solve_mixed(cab.rp, cab.ci, cab.vals, cab.b, rtol=1e-10, maxiter=50000,
                                                   inner_rtol=None if extra else 1e-4,
                                                   flags=hz.PRECOND_JACOBI | hz.X0_ZERO | extra)
                torch.cuda.synchronize()
                print(what, label, "ms", round(1e3 * (time.perf_counter() - t0), 2), info, flush=True)
    elif what == "solve-cylinder":
        import workloads as W

        A, b, _ = W.config_cylinder()
        rp, ci, v, bd = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (A.row_ptr, A.col_idx, A.vals, b))
        for _ in range(steps):
            t0 = time.perf_counter()
            _, info = hz.zbicgstab_solve(rp, ci, v, bd, rtol=1e-10, maxiter=50000, flags=hz.PRECOND_JACOBI | hz.X0_ZERO)
            torch.cuda.synchronize()
            print(what, "ms", round(1e3 * (time.perf_counter() - t0), 2), info, flush=True)
    elif what in ("sweep-explicit", "sweep-kmb"):
        # 200 iterations of the 64-frequency batch, every system still active (they need 1,249 or more)
        import workloads as W

        A, vals, rhs, ks, sw = W.config_freq_sweep(B=64)
        n, nnz, B = A.n, A.nnz, 64
        rp, ci = torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col_idx).to(dev)
        Bm = torch.from_numpy(np.ascontiguousarray(rhs.T)).to(dev)
        X = torch.zeros_like(Bm)
        flags = hz.PRECOND_JACOBI | hz.X0_ZERO
        if what == "sweep-explicit":
            V = torch.from_numpy(np.ascontiguousarray(vals.T)).to(dev)
            ws = torch.empty(hz.zbicgstab_batched_workspace_bytes(B, n, nnz, flags) + 256, dtype=torch.uint8,
                             device=dev)
            run = lambda: hz.zbicgstab_solve_batched(rp, ci, V, Bm, x=X, rtol=1e-10, maxiter=200,  # noqa: E731
                                                     flags=flags, ws=ws)
        else:
            Kd, Md, Bd = (torch.from_numpy(sw[k]).to(dev) for k in ("K", "M", "B"))
            ws = torch.empty(hz.zbicgstab_sweep_workspace_bytes(B, n, nnz, flags) + 256, dtype=torch.uint8,
                             device=dev)
            run = lambda: hz.zbicgstab_solve_sweep(rp, ci, Kd, Md, Bd, ks, Bm, x=X, rtol=1e-10,  # noqa: E731
                                                   maxiter=200, flags=flags, ws=ws)
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = run()
            torch.cuda.synchronize()
            print(what, "ms per iteration", round((time.perf_counter() - t0) * 1e3 / 200, 4),
                  "active", sum(i["status"] == 1 for i in infos), flush=True)
    elif what == "adjoint-cylinder":
        for _ in range(steps):
            print(what, json.dumps(adjoint_cylinder(hz, torch, dev)), flush=True)
    elif what == "stream":
        print(what, json.dumps(stream_ceiling(hz, torch, dev)), flush=True)
    elif what == "blas1":
        # zdotc, dznrm2 and zaxpy at n = 1.5e7 (HBM-bound) and 209,777 (launch-bound), 20 eager calls each per step
        rng = np.random.default_rng(5)
        for n in (15_000_000, 209_777):
            x = torch.from_numpy(rng.standard_normal(2 * n).view(np.complex128)).to(dev)
            y = torch.from_numpy(rng.standard_normal(2 * n).view(np.complex128)).to(dev)
            d = torch.empty((), dtype=torch.complex128, device=dev)
            nr = torch.empty((), dtype=torch.float64, device=dev)
            for _ in range(steps):
                for _ in range(20):
                    hz.zdotc(x, y, out=d)
                for _ in range(20):
                    hz.dznrm2(x, out=nr)
                for _ in range(20):
                    hz.zaxpy(1e-3 + 0j, x, y)
                torch.cuda.synchronize()
            print(what, n, complex(d.cpu()), float(nr.cpu()), flush=True)
            del x, y
    else:
        raise SystemExit(f"unknown profile target {what}")


# ---------------------------------------------------------------- main


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--spmv-reps", type=int, default=30)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cache", default=None, help="directory to keep generated workloads in (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--profile", default=None,
                    help="spmv-cabin | spmv-cabin-rows | spmv-cabin-given | spmv-cabin-given-tiles | spmv-cabin-planned | spmv-cabin-ell | solve-cabin | solve-cabin-l8 | spmv-cylinder | spmv-cylinder-rows | solve-cabin-mixed | solve-cylinder | "
                         "sweep-explicit | sweep-kmb | "
                         "adjoint-cylinder | stream | blas1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline step only (no secondary sections)")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched cube solves")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-frequency shared-pattern batch")
    ap.add_argument("--no-blas1", action="store_true", help="skip the standalone zdotc/dznrm2/zaxpy sizes")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the cylinder backward pass")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the solve is not sharded).",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return
    if args.profile:
        profile(args.profile, args.steps, args.cache)
        return

    import torch

    import paper_2112_06465_amd as hz

    dev = torch.device("cuda:0")
    cab = Cabin(hz, torch, dev, args.cache)
    n, nnz = cab.n, cab.nnz
    loop = ColdLoop(torch, lambda r: hz.csr_zspmv(*r), cab.replicas(torch, level=True), args.spmv_reps)
    yv, zv = torch.empty_like(cab.x), cab.x.clone()
    dotout = torch.empty((), dtype=torch.complex128, device=dev)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    ws = hz.workspace(n, nnz, flags, dev)
    xs = torch.zeros_like(cab.b)

    def step(record):
        with PinnedForm(CABIN_FORM):
            loop.enqueue()
        hz.zdotc(cab.x, yv, out=dotout)
        hz.zaxpy(0.7 - 0.3j, cab.x, zv)
        _, sinfo = hz.zbicgstab_solve(cab.rp, cab.ci, cab.vals, cab.b, x=xs, rtol=args.tol, maxiter=50000,
                                      flags=flags, ws=ws)
        return sinfo, (loop.us() if record else None)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    step_ms, spmv_us, infos = [], [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sinfo, us = step(True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        spmv_us.append(us)
        infos.append(sinfo)
    total_s = time.perf_counter() - t_start

    its = [i["iterations"] for i in infos]
    step_bytes = [(args.spmv_reps + 1) * spmv_bytes(n, nnz) + 80 * n + solve_bytes(n, nnz, it) for it in its]
    us = float(np.mean(spmv_us))
    gbs = spmv_bytes(n, nnz) / (us * 1e-6) / 1e9
    kernel = spmv_kernel_name(CABIN_FORM)
    ceiling = stream_ceiling(hz, torch, dev)
    ceil_gbs = ceiling["read_2GiB"]["GBs"]
    true_rr = host_relres(cab.A, xs.cpu().numpy(), cab.b_np)

    out = {
        "metric": "zSpMV HBM GB/s (% of peak); BiCGStab time-to-1e-10, mixed vs FP64, 1 MI355X",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_s * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded P1 FEM cabin, random node numbering, point source + noise RHS)",
        "config": {
            "workload": f"cabin P1 FEM h=0.012 k=40, randomly numbered (n={n}, nnz={nnz}): per step "
                        f"{args.spmv_reps + 1} cold zSpMV of the level-set renumbered matrix + zdotc + zaxpy + "
                        f"Jacobi-BiCGStab to {args.tol:g} in the caller's numbering",
            "n": n,
            "nnz": nnz,
            "value_definition": "zSpMV algorithmic bytes (20 nnz + 36 n + 4) / HIP-event average launch time of "
                                "the cold products of the timed steps",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": read_traffic("zspmv_cabin_pmc.md", kernel),
            "algorithmic_bytes_per_launch": spmv_bytes(n, nnz),
            "avg_launch_us": round(us, 3),
            "measured_read_ceiling_GBs": ceil_gbs,
            "frac_of_measured_ceiling": round(gbs / ceil_gbs, 4),
            "target_frac": 0.70,
            "cache": f"cold: launches alternate between {CABIN_REPLICAS} replicas (> 256 MB Infinity Cache)",
        },
        "step": {
            "algorithmic_GBs": round(sum(step_bytes) / total_s / 1e9, 1),
            "solve_iterations": its[-1],
            "solve_status": infos[-1]["status"],
            "solve_renumbered": infos[-1]["renumbered"],
            "relres_recursive": infos[-1]["relres_recursive"],
            "relres_true_gpu": infos[-1]["relres_true"],
            "relres_true_host": true_rr,
            "step_ms": [round(s, 3) for s in step_ms],
            "spmv_us_per_step": [round(u, 3) for u in spmv_us],
        },
        "stream_ceiling": ceiling,
    }
    if not args.no_extras:
        out["spmv_cabin"] = spmv_cabin(hz, torch, dev, cab)
        out["spmv_cylinder_cold"] = spmv_cylinder(hz, torch, dev)
        if not args.no_time_to_tol:
            import workloads as W

            out["time_to_tol"] = []
            all_runs = ["fp64", "mixed", "mixed_reliable", "bicgstab_l8", "tfqmr"]
            A1, b1, _ = W.config_cylinder()
            up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
            out["time_to_tol"].append(time_solves(hz, torch, dev, "cylinder, impedance on the whole boundary", A1,
                                                  b1, up(A1.row_ptr), up(A1.col_idx), up(A1.vals), 1e-10, all_runs))
            A1c, b1c, _ = W.config_cylinder(robin="caps")
            out["time_to_tol"].append(time_solves(hz, torch, dev, "cylinder, Robin on the end caps only", A1c, b1c,
                                                  up(A1c.row_ptr), up(A1c.col_idx), up(A1c.vals), 1e-8,
                                                  ["fp64", "bicgstab_l8", "tfqmr"], maxiter=20000, maxcycles=4000))
            out["time_to_tol"].append(time_solves(hz, torch, dev, "cabin", cab.A, cab.b_np, cab.rp, cab.ci,
                                                  cab.vals, 1e-10, all_runs + ["fp64_caller_order"]))
        if not args.no_adjoint:
            out["adjoint"] = adjoint_cylinder(hz, torch, dev)
        if not args.no_batched:
            out["batched"] = batched_cubes(hz, torch, dev)
        if not args.no_sweep:
            out["batched_sweep"] = batched_sweep(hz, torch, dev)
        if not args.no_blas1:
            out["blas1"] = blas1(hz, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cab)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
