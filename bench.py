#!/usr/bin/env python3
"""Benchmark of the Helmholtz BiCGStab hot path on one MI355X.

One step = the whole hot path on the cylinder workload (P1 Kuhn-tet FEM,
radius 1, length 4, h = 0.04, k = 20: n = 209,777, nnz = 3,048,433):
  1. R standalone complex128 SpMVs (csr_zspmv), cycling through 6 replicas
     of the matrix and vectors (6 x 72 MB > the 256 MB Infinity Cache, so
     every launch starts cold), bracketed by one pair of HIP events on the
     launch stream;
  2. one zdotc and one zaxpy on the n-vectors;
  3. one Jacobi-BiCGStab solve of A x = b to ||r||/||b|| <= 1e-8.

``value`` = algorithmic HBM bytes of every kernel of the step / step time
(GB/s).  The algorithmic byte model (each array element moved once):
  SpMV                 20 nnz + 36 n + 4
  zdotc / zaxpy        32 n / 48 n
  BiCGStab iteration   40 nnz + 280 n   (three fused kernels, Jacobi folded)
  solve set-up/finish  76 nnz + 168 n   (diagonal, column scaling, init,
                                          un-scaling, true residual)
``roofline`` reports the standalone zSpMV kernel against the 8 TB/s HBM
peak; its duration is the HIP-event average over the timed region.
``cpu_baseline`` times the plain C oracle on a bounded sample of the same
work, single-threaded, on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --calib-copy       (plain copy for counter scaling)
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
N_REPLICAS = 6
PROFILES = os.path.join(ROOT, "profiles")


def spmv_kernel_name(form, L):
    """Name of the standalone zSpMV kernel for a form ("rows" / "tiles") and lane count."""
    if form == "tiles":
        return "hz::k_spmv_tile<double>"
    U = 4 if L <= 4 else (2 if L == 8 else 1)
    return f"hz::k_spmv_pipe<double, {L}, {U}>"


def spmv_bytes(n, nnz):
    return 20 * nnz + 36 * n + 4


def solve_bytes(n, nnz, iterations):
    return iterations * (40 * nnz + 280 * n) + 76 * nnz + 168 * n


def kernel_source_hash() -> str:
    """Hash of the device source of the standalone SpMV kernels (hz_spmv.hpp and hz_kernels.hpp)."""
    h = hashlib.sha256()
    for f in ("hz_spmv.hpp", "hz_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2112_06465_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if current."""
    path = os.path.join(PROFILES, "zspmv_cylinder_pmc.md")
    try:
        txt = open(path).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel source hash:\s*`?([0-9a-f]{16})", txt)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    m_bytes = re.search(r"HBM bytes per launch \(scaled\), `" + re.escape(kernel) + r"`:\s*([0-9.eE+]+)", txt)
    return float(m_bytes.group(1)) if m_bytes else None


def cpu_baseline(A, b, x_spmv, spmv_reps=31, maxiter=20000):
    """Time the oracle (single thread) on one step's work: the products, zdotc, zaxpy and the whole solve.

    On the cylinder this is about 10 s of CPU time (the solve to 1e-8 takes ~1,200 iterations), the bounded
    sample the bench line reports beside the GPU figure.
    """
    import oracle as O

    n, nnz = A.n, A.nnz
    t0 = time.perf_counter()
    for _ in range(spmv_reps):
        O.zspmv(A, x_spmv)
    O.zdotc(x_spmv, b)
    O.zaxpy(0.7 - 0.3j, x_spmv, b)
    _, info = O.zbicgstab(A, b, tol=1e-8, maxiter=maxiter, jacobi=True)
    dt = time.perf_counter() - t0
    it = info["iterations"]
    # bytes of the same model as the GPU step
    nbytes = spmv_reps * spmv_bytes(n, nnz) + 32 * n + 48 * n + solve_bytes(n, nnz, it)
    return {
        "value": nbytes / dt / 1e9,
        "unit": "GB/s",
        "cores": O.threads_used(),
        "kind": "oracle",
        "sample": f"one step on the cylinder n={n} nnz={nnz}: {spmv_reps} zSpMV + zdotc + zaxpy + Jacobi-BiCGStab "
        f"to 1e-8 ({it} iterations), single thread, {dt:.1f} s on '{O.cpu_model()}'",
        "seconds": dt,
    }


def time_to_tol(hz, torch, dev, name, rp, ci, vals, b, A, tol=1e-10, caller_order_too=False):
    """Wall time of a Jacobi-BiCGStab solve to tol: plain FP64 vs complex64-inner refinement."""
    import oracle as O

    n, nnz = A.n, A.nnz
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    ws = hz.workspace(n, nnz, flags, dev)
    wsm = hz.mixed_workspace(n, nnz, flags, dev)
    wsl = torch.empty(hz.zbicgstabl_workspace_bytes(n, nnz, 8, flags) + 256, dtype=torch.uint8, device=dev)
    wsq = torch.empty(hz.ztfqmr_workspace_bytes(n, nnz, flags) + 256, dtype=torch.uint8, device=dev)
    x = torch.zeros_like(b)
    res = {"workload": f"{name} (n={n}, nnz={nnz})", "tol": tol}
    runs = [
        ("fp64", lambda: hz.zbicgstab_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=50000, flags=flags, ws=ws)),
        ("mixed", lambda: hz.zbicgstab_solve_mixed(rp, ci, vals, b, x=x, rtol=tol, inner_rtol=1e-4, maxiter=50000,
                                                   flags=flags, ws=wsm)),
        ("mixed_reliable", lambda: hz.zbicgstab_solve_mixed(rp, ci, vals, b, x=x, rtol=tol, maxiter=50000,
                                                            flags=flags | hz.RELIABLE, ws=wsm)),
        # BiCGstab(8), the paper's second solver: iterations are cycles of 8 Bi-CG steps (16 products)
        ("bicgstab_l8", lambda: hz.zbicgstabl_solve(rp, ci, vals, b, x=x, ell=8, rtol=tol, maxcycles=5000,
                                                    flags=flags, ws=wsl)),
        # TFQMR, the paper's third solver: two products per iteration, stopped on the quasi-residual bound
        ("tfqmr", lambda: hz.ztfqmr_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=50000, flags=flags, ws=wsq)),
    ]
    if caller_order_too:
        # the same FP64 solve kept in the caller's numbering (no level-set renumbering)
        runs.append(("fp64_caller_order", lambda: hz.zbicgstab_solve(rp, ci, vals, b, x=x, rtol=tol, maxiter=50000,
                                                                     flags=flags | hz.NO_REORDER, ws=ws)))
    for label, fn in runs:
        fn()  # warm-up (also the JIT of nothing: the library is precompiled)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        xh = x.cpu().numpy()
        bh = b.cpu().numpy()
        rr = float(np.linalg.norm(bh - O.zspmv(A, xh)) / np.linalg.norm(bh))
        res[label] = {"ms": round(ms, 3), "iterations": info["iterations"], "outer_steps": info["outer_steps"],
                      "status": info["status"], "renumbered": info["renumbered"], "relres_true_oracle_spmv": rr}
        if label == "fp64":
            x64 = xh.copy()
        else:
            res[label]["rel_err_vs_fp64"] = float(np.linalg.norm(xh - x64) / np.linalg.norm(x64))
    res["mixed_speedup"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
    res["mixed_reliable_speedup"] = round(res["fp64"]["ms"] / res["mixed_reliable"]["ms"], 3)
    res["bicgstab_l8_speedup"] = round(res["fp64"]["ms"] / res["bicgstab_l8"]["ms"], 3)
    res["tfqmr_speedup"] = round(res["fp64"]["ms"] / res["tfqmr"]["ms"], 3)
    return res


def spmv_cabin(hz, torch, dev, A, rp, ci, vals, reps=10):
    """zSpMV on the cabin (403 MB, beyond the Infinity Cache) in the given random numbering and in level sets."""
    n, nnz = A.n, A.nnz
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(dev)
    y = torch.empty_like(x)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def timed(r, c, v, xx):
        for _ in range(2):
            hz.csr_zspmv(r, c, v, xx, y)
        ev[0].record()
        for _ in range(reps):
            hz.csr_zspmv(r, c, v, xx, y)
        ev[1].record()
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        gbs = spmv_bytes(n, nnz) / (us * 1e-6) / 1e9
        return {"us": round(us, 2), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}

    res = {"workload": f"cabin (n={n}, nnz={nnz}), algorithmic bytes {spmv_bytes(n, nnz)}, {reps} launches"}
    res["given_numbering"] = timed(rp, ci, vals, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm, inv, level = hz.csr_level_order(rp, ci)
    rp2, ci2, v2 = hz.csr_zpermute(rp, ci, vals, perm, inv)
    torch.cuda.synchronize()
    res["analysis_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    res["levels"] = int(level.max().item()) + 1
    xp = x[perm.long()].contiguous()
    res["level_sets"] = timed(rp2, ci2, v2, xp)
    tune = hz.autotune_spmv(rp2, ci2, v2, xp, details=True)
    res["level_sets_tuned"] = dict(timed(rp2, ci2, v2, xp), form=tune["form"], lanes=tune["form_lanes"])
    # the same renumbered matrix in ELL (its longest row: 15 entries against a mean of 14.6)
    ell = hz.csr_to_hyb(rp2, ci2, v2, K="ell")
    for _ in range(2):
        hz.hyb_zspmv(ell, xp, y)
    ev[0].record()
    for _ in range(reps):
        hz.hyb_zspmv(ell, xp, y)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    gbs = spmv_bytes(n, nnz) / (us * 1e-6) / 1e9
    res["level_sets_ell"] = {"us": round(us, 2), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                             "K": ell["K"]}
    return res


def spmv_formats(hz, torch, dev, A, rp, ci, vals, replicas=6, reps=30):
    """Cold zSpMV of the cylinder in ELL (HYB at the longest row) and SELL-64-1, beside CSR.

    The same replica cycling as the roofline loop (every launch reads cold data); GB/s on the CSR byte model, so
    the figures compare the operation, and each format's stored bytes beside them.
    """
    n, nnz = A.n, A.nnz
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    res = {"workload": f"cylinder (n={n}, nnz={nnz}), {replicas} replicas, {reps} launches"}
    for label, conv, prod, stored in (
        ("ell", lambda r, c, v: hz.csr_to_hyb(r, c, v, K="ell"), hz.hyb_zspmv,
         lambda f: 20 * f["K"] * n + 32 * n),
        ("sell_64_1", lambda r, c, v: hz.csr_to_sell(r, c, v, C=64, sigma=1, t=1), hz.sell_zspmv,
         lambda f: 20 * f["col"].numel() + 4 * n + 8 * f["chunk_ptr"].numel() + 32 * n),
    ):
        reps_ = [(conv(rp.clone(), ci.clone(), vals.clone()), x.clone(), torch.empty_like(x)) for _ in range(replicas)]
        for f, xx, yy in reps_:
            prod(f, xx, yy)
        ev[0].record()
        for k in range(reps):
            f, xx, yy = reps_[k % replicas]
            prod(f, xx, yy)
        ev[1].record()
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        gbs = spmv_bytes(n, nnz) / (us * 1e-6) / 1e9
        res[label] = {"us": round(us, 2), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                      "stored_bytes": int(stored(reps_[0][0]))}
        del reps_
        torch.cuda.empty_cache()
    return res


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
    import oracle as O
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
    # warm-up: two iterations of each form
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
    # the same sweep from the three real matrices (K - k^2 M + i k B formed in the kernels)
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
    Xkh = Xk.cpu().numpy()
    rr_k = max(float(np.linalg.norm(rhs[j] - O.zspmv(A.with_vals(vals[j]), Xkh[:, j])) / np.linalg.norm(rhs[j]))
               for j in range(B))
    Xh = X.cpu().numpy()
    rr_b = max(float(np.linalg.norm(rhs[j] - O.zspmv(A.with_vals(vals[j]), Xh[:, j])) / np.linalg.norm(rhs[j]))
               for j in range(B))
    rr_s = max(float(np.linalg.norm(rhs[j] - O.zspmv(A.with_vals(vals[j]), xs[j].cpu().numpy()))
                     / np.linalg.norm(rhs[j])) for j in range(B))
    its = [i["iterations"] for i in binfo]
    return {
        "workload": f"{B} wavenumbers k~U[10,40] on the cylinder pattern (n={n}, nnz={nnz}), Jacobi, tol {tol:g}",
        "batched_ms": round(t_b * 1e3, 3), "sequential_ms": round(t_s * 1e3, 3), "speedup": round(t_s / t_b, 3),
        "from_K_M_B": {"ms": round(t_k * 1e3, 3), "speedup_vs_sequential": round(t_s / t_k, 3),
                       "iterations_min_max": [min(i["iterations"] for i in kinfo), max(i["iterations"] for i in kinfo)],
                       "all_ok": all(i["status"] == 0 for i in kinfo), "max_relres_true_oracle_spmv": rr_k},
        "iterations_min_max": [min(its), max(its)],
        "iterations_sequential_min_max": [min(i["iterations"] for i in sinfo), max(i["iterations"] for i in sinfo)],
        "all_ok": all(i["status"] == 0 for i in binfo) and all(i["status"] == 0 for i in sinfo),
        "max_relres_true_oracle_spmv": {"batched": rr_b, "sequential": rr_s},
        # each system streams its own values and vectors while it runs; indices once per iteration
        "batched_algorithmic_GBs": round((sum(its) * (32 * nnz + 304 * n) + max(its) * (8 * nnz + 8 * n)) / t_b / 1e9,
                                         1),
    }


def batched_cubes(hz, torch, dev, B=32, tol=1e-8):
    """32 independent 7-point cubes (N ~ U{16..64}, own k): one batched solve vs 32 sequential solves."""
    import oracle as O
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

    def run_batched():
        return hz.zbicgstab_solve_varbatch(ro, rp, ci, vv, bb, x=xb, rtol=tol, maxiter=50000, flags=flags, ws=wsb)

    def run_sequential():
        return [hz.zbicgstab_solve(*s, x=x, rtol=tol, maxiter=50000, flags=flags, ws=wss) for s, x in zip(singles, xs)]

    res = {"workload": f"{B} cubes N~U{{16..64}} (sum n={int(row_off[-1])}, nnz={nnz_off}), unpreconditioned, tol {tol:g}"}
    for label, fn in (("batched", run_batched), ("sequential", run_sequential)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        res[label + "_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        if label == "batched":
            infos = out[1]
            res["iterations_min_max"] = [min(i["iterations"] for i in infos), max(i["iterations"] for i in infos)]
            res["all_ok"] = all(i["status"] == 0 for i in infos)
            xh = xb.cpu().numpy()
            res["max_relres_true_oracle_spmv"] = max(
                float(np.linalg.norm(b - O.zspmv(A, xh[row_off[j]:row_off[j + 1]])) / np.linalg.norm(b))
                for j, (A, b) in enumerate(systems)
            )
    res["speedup"] = round(res["sequential_ms"] / res["batched_ms"], 3)
    return res


def calib_copy():
    import torch

    nbytes = 512 * 2**20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--spmv-reps", type=int, default=30)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--no-cabin", action="store_true", help="skip FP64 vs mixed to 1e-10 on the cabin")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched cube solve")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-frequency shared-pattern batch")
    ap.add_argument("--no-blas1", action="store_true", help="skip the standalone zdotc/dznrm2/zaxpy sizes")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the solve is not sharded).",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return

    import torch

    import paper_2112_06465_amd as hz
    import workloads as W

    dev = torch.device("cuda:0")
    A, b_np, info = W.config_cylinder()
    n, nnz = A.n, A.nnz
    rng = np.random.default_rng(0)
    x_np = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    vals = torch.from_numpy(A.vals).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    xv = torch.from_numpy(x_np).to(dev)
    yv = torch.empty_like(xv)
    zv = xv.clone()
    # launch shapes for this matrix, tuned outside the timed region (the solver's lane count). The cold
    # standalone loop below runs on replicas (other index arrays for the handle) with the built-in rule's
    # form pinned: vector rows at the smallest power of two >= half the mean row length. The tuner's warm
    # timings of the candidates near that one differ by less than run-to-run noise, and a fixed kernel
    # keeps this line and the committed profiles about the same kernel.
    tune = hz.autotune_spmv(rp, ci, vals, xv, details=True)
    lanes = tune["lanes"]
    sp_form, sp_lanes = "rows", 2
    while sp_lanes < 64 and 2 * sp_lanes < nnz / n:
        sp_lanes *= 2
    xs = torch.zeros_like(b)
    flags = hz.PRECOND_JACOBI | hz.X0_ZERO
    ws = hz.workspace(n, nnz, flags, dev)
    reps = [(rp, ci, vals, xv, yv)] + [
        (rp.clone(), ci.clone(), vals.clone(), xv.clone(), torch.empty_like(yv)) for _ in range(N_REPLICAS - 1)
    ]
    dotout = torch.empty((), dtype=torch.complex128, device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def step(record):
        spmv_ms = []
        os.environ["HZ_SPMV_FORM"], os.environ["HZ_SPMV_LANES"] = sp_form, str(sp_lanes)
        # one launch enqueued ahead of the start event, so the GPU is busy when the timed region opens and
        # the host's first call is not counted as idle time (the stream is idle after the previous step)
        hz.csr_zspmv(*reps[N_REPLICAS - 1])
        ev[0].record()
        for r in range(args.spmv_reps):
            hz.csr_zspmv(*reps[r % N_REPLICAS])
        ev[1].record()
        del os.environ["HZ_SPMV_FORM"], os.environ["HZ_SPMV_LANES"]
        hz.zdotc(xv, yv, out=dotout)
        hz.zaxpy(0.7 - 0.3j, xv, zv)
        _, sinfo = hz.zbicgstab_solve(rp, ci, vals, b, x=xs, rtol=args.tol, maxiter=20000, flags=flags, ws=ws)
        if record:
            torch.cuda.synchronize()
            spmv_ms = [ev[0].elapsed_time(ev[1]) / args.spmv_reps]
        return sinfo, spmv_ms

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    step_ms, spmv_all, infos = [], [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sinfo, spmv_ms = step(True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        spmv_all += spmv_ms
        infos.append(sinfo)
    total_s = time.perf_counter() - t_start

    its = [i["iterations"] for i in infos]
    step_bytes = [
        (args.spmv_reps + 1) * spmv_bytes(n, nnz) + 32 * n + 48 * n + solve_bytes(n, nnz, it) for it in its
    ]
    value = sum(step_bytes) / total_s / 1e9
    spmv_avg_s = float(np.mean(spmv_all)) / 1e3
    spmv_gbs = spmv_bytes(n, nnz) / spmv_avg_s / 1e9
    traffic = read_traffic(spmv_kernel_name(sp_form, sp_lanes))

    # correctness of the last solve, checked on the host with the oracle
    import oracle as O

    x_host = xs.cpu().numpy()
    true_rr = float(np.linalg.norm(b_np - O.zspmv(A, x_host)) / np.linalg.norm(b_np))

    out = {
        "metric": "zSpMV HBM GB/s (% of peak); BiCGStab time-to-1e-10, mixed vs FP64, 1 MI355X",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_s * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded P1 FEM cylinder, point source + noise RHS)",
        "config": {
            "workload": f"cylinder P1 FEM h=0.04 k=20 impedance boundary (n={n}, nnz={nnz}): "
            f"{args.spmv_reps + 1} cold zSpMV + zdotc + zaxpy + Jacobi-BiCGStab to {args.tol:g}",
            "n": n,
            "nnz": nnz,
            "value_definition": "algorithmic HBM bytes of all kernels in a step / wall time of the steps",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": spmv_kernel_name(sp_form, sp_lanes),
            "form": sp_form,
            "lanes_per_row": sp_lanes,
            "achieved": round(spmv_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": spmv_bytes(n, nnz),
            "avg_launch_us": round(spmv_avg_s * 1e6, 3),
            "cache": f"cold: launches cycle through {N_REPLICAS} replicas (> 256 MB Infinity Cache)",
        },
        "solve": {
            "iterations": its[-1],
            "status": infos[-1]["status"],
            "relres_recursive": infos[-1]["relres_recursive"],
            "relres_true_gpu": infos[-1]["relres_true"],
            "relres_true_oracle_spmv": true_rr,
            "step_ms": [round(s, 3) for s in step_ms],
        },
    }
    out["spmv_formats"] = spmv_formats(hz, torch, dev, A, rp, ci, vals)
    if not args.no_time_to_tol:
        out["time_to_tol"] = [time_to_tol(hz, torch, dev, "cylinder", rp, ci, vals, b, A)]
        if not args.no_cabin:
            Ac, bc, _ = W.config_cabin()
            rpc, cic, vc = (torch.from_numpy(a).to(dev) for a in (Ac.row_ptr, Ac.col_idx, Ac.vals))
            out["spmv_cabin"] = spmv_cabin(hz, torch, dev, Ac, rpc, cic, vc)
            t = time_to_tol(hz, torch, dev, "cabin", rpc, cic, vc, torch.from_numpy(bc).to(dev), Ac,
                            caller_order_too=True)
            out["time_to_tol"].append(t)
    if not args.no_batched:
        out["batched"] = batched_cubes(hz, torch, dev)
    if not args.no_sweep:
        out["batched_sweep"] = batched_sweep(hz, torch, dev)
    if not args.no_blas1:
        out["blas1"] = blas1(hz, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, b_np, x_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
