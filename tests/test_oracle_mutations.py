"""The oracle's pins catch plausible mistakes planted in a scratch copy of the oracle (CPU only).

Each mutant copies oracle/, workloads/ and the pin tests into a temporary
directory, changes one line of the oracle (the C solvers, the BiCGstab(l), TFQMR or
storage-format module), and runs the pins of that part there: they must fail.  The repository's own oracle is never modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "dot_without_conjugation": (
        "krylov.c",
        "static CPLX cmulc(CPLX a, CPLX b) { return cmk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }",
        "static CPLX cmulc(CPLX a, CPLX b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }",
    ),
    "complex_product_sign": (
        "krylov.c",
        "return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }",
        "return cmk(a.re * b.re + a.im * b.im, a.re * b.im + a.im * b.re); }",
    ),
    "spmv_wrong_operand_index": (
        "krylov.c",
        "acc = cadd(acc, cmul(vals[p], x[col_idx[p]]));",
        "acc = cadd(acc, cmul(vals[p], x[i]));",
    ),
    "beta_ratio_inverted": (
        "krylov.c",
        "CPLX beta = cmul(cdiv(rho, rho_prev), cdiv(alpha, omega));",
        "CPLX beta = cmul(cdiv(rho_prev, rho), cdiv(alpha, omega));",
    ),
    "half_step_drops_update": (
        "krylov.c",
        "                x[i] = cadd(x[i], cmul(alpha, phat[i]));\n            status = OR_OK;",
        "                x[i] = x[i];\n            status = OR_OK;",
    ),
    "omega_conjugated": (
        "krylov.c",
        "omega = cdiv(FN(dotc)(n, t, s), tt);",
        "omega = cdiv(FN(dotc)(n, s, t), tt);",
    ),
    "axpy_drops_y": ("krylov.c", "y[i] = cadd(cmul(alpha, x[i]), y[i]);", "y[i] = cmul(alpha, x[i]);"),
    "norm_drops_imaginary": ("krylov.c", "acc += x[i].re * x[i].re + x[i].im * x[i].im;", "acc += x[i].re * x[i].re;"),
    "jacobi_not_inverted": ("krylov.c", "dinv[i] = cdiv(cmk(1, 0), d);", "dinv[i] = d;"),
    "gradient_without_conjugation": (
        "refine.c",
        "grad_vals[p].re = -(l.re * xc.re + l.im * xc.im);\n            grad_vals[p].im = -(l.im * xc.re - l.re * xc.im);",
        "grad_vals[p].re = -(l.re * xc.re - l.im * xc.im);\n            grad_vals[p].im = -(l.im * xc.re + l.re * xc.im);",
    ),
    "transpose_without_conjugation": ("refine.c", "t_vals[q].im = -vals[p].im;", "t_vals[q].im = vals[p].im;"),
    "refinement_drops_scale": (
        "refine.c",
        "x[i].re = x[i].re + rn * (double)d32[i].re;",
        "x[i].re = x[i].re + (double)d32[i].re;",
    ),
    # BiCGstab(l) (oracle/bicgstabl.py), against its own pins
    "bicgstabl_beta_inverted": (
        "bicgstabl.py",
        "beta = alpha * rho1 / rho0",
        "beta = alpha * rho0 / rho1",
        "tests/test_oracle_bicgstabl_pins.py",
    ),
    "bicgstabl_direction_sign": (
        "bicgstabl.py",
        "uhat[i] = rhat[i] - beta * uhat[i]",
        "uhat[i] = rhat[i] + beta * uhat[i]",
        "tests/test_oracle_bicgstabl_pins.py",
    ),
    "bicgstabl_x_update_shifted_basis": (
        "bicgstabl.py",
        "y = y + np.column_stack(rhat[:ell]) @ g",
        "y = y + np.column_stack(rhat[1:]) @ g",
        "tests/test_oracle_bicgstabl_pins.py",
    ),
    "bicgstabl_omega_from_first_coefficient": (
        "bicgstabl.py",
        "omega = complex(g[-1])",
        "omega = complex(g[0])",
        "tests/test_oracle_bicgstabl_pins.py",
    ),
    "bicgstabl_rho_not_negated": (
        "bicgstabl.py",
        "rho0 = -omega * rho0",
        "rho0 = omega * rho0",
        "tests/test_oracle_bicgstabl_pins.py",
    ),
    # TFQMR (oracle/tfqmr.py), against its own pins
    "tfqmr_beta_inverted": ("tfqmr.py", "beta = rho_new / rho", "beta = rho / rho_new", "tests/test_oracle_tfqmr_pins.py"),
    "tfqmr_d_drops_eta": (
        "tfqmr.py",
        "d = u + (theta * theta / alpha) * eta * d",
        "d = u + (theta * theta / alpha) * d",
        "tests/test_oracle_tfqmr_pins.py",
    ),
    "tfqmr_tau_without_c": ("tfqmr.py", "tau = tau * theta * c", "tau = tau * theta", "tests/test_oracle_tfqmr_pins.py"),
    "tfqmr_v_update_sign": (
        "tfqmr.py",
        "v = Au + beta * (Au_odd + beta * v_prev)",
        "v = Au + beta * (Au_odd - beta * v_prev)",
        "tests/test_oracle_tfqmr_pins.py",
    ),
    "tfqmr_eta_without_c_squared": ("tfqmr.py", "eta = c * c * alpha", "eta = c * alpha", "tests/test_oracle_tfqmr_pins.py"),
    # reliable updates (oracle/reliable.py), against their own pins
    "reliable_update_drops_scale": (
        "reliable.py",
        "x = x + bn * (dinv.astype(np.complex128) * y.astype(np.complex128))",
        "x = x + (dinv.astype(np.complex128) * y.astype(np.complex128))",
        "tests/test_oracle_reliable_pins.py",
    ),
    "reliable_residual_not_replaced": (
        "reliable.py",
        "            r = (r64 / bn).astype(inner)\n            r_ref = float(np.linalg.norm(r.astype(np.complex128)))\n    if status",
        "            r_ref = float(np.linalg.norm(r.astype(np.complex128)))\n    if status",
        "tests/test_oracle_reliable_pins.py",
    ),
    "reliable_omega_conjugated": (
        "reliable.py",
        "omega = _dot(t, s) / tt",
        "omega = _dot(s, t) / tt",
        "tests/test_oracle_reliable_pins.py",
    ),
    "reliable_jacobi_not_inverted": (
        "reliable.py",
        "dinv = (1.0 / d).astype(inner)",
        "dinv = d.astype(inner)",
        "tests/test_oracle_reliable_pins.py",
    ),
    "reliable_y_drops_omega_term": (
        "reliable.py",
        "y = (y + c(alpha) * p + c(omega) * s).astype(inner)",
        "y = (y + c(alpha) * p).astype(inner)",
        "tests/test_oracle_reliable_pins.py",
    ),
    # storage formats (oracle/formats.py), against their own pins
    "sell_sorted_ascending": (
        "formats.py",
        "rows.sort(key=lambda i: -lens[i])",
        "rows.sort(key=lambda i: lens[i])",
        "tests/test_oracle_formats_pins.py",
    ),
    "sell_lanes_transposed": (
        "formats.py",
        "q = int(chunk_ptr[c]) + (k // t) * C * t + r * t + (k % t)\n            col[q]",
        "q = int(chunk_ptr[c]) + (k // t) * C * t + r + (k % t) * C\n            col[q]",
        "tests/test_oracle_formats_pins.py",
    ),
    "sell_width_not_rounded_to_lanes": (
        "formats.py",
        "w = -(-longest // t) * t",
        "w = longest",
        "tests/test_oracle_formats_pins.py",
    ),
    "ell_row_major": (
        "formats.py",
        "col[k * n + i] = A.col_idx[lo + k]\n                val[k * n + i] = A.vals[lo + k]",
        "col[i * K + k] = A.col_idx[lo + k]\n                val[i * K + k] = A.vals[lo + k]",
        "tests/test_oracle_formats_pins.py",
    ),
    "hyb_width_strict": (
        "formats.py",
        "if np.count_nonzero(lens >= k) >= need:",
        "if np.count_nonzero(lens >= k) > need:",
        "tests/test_oracle_formats_pins.py",
    ),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    fname, old, new = MUTANTS[name][:3]
    pins = MUTANTS[name][3] if len(MUTANTS[name]) > 3 else "tests/test_oracle_pins.py"
    work = tmp_path / "repo"
    work.mkdir()
    for d in ("oracle", "workloads", "tests"):
        shutil.copytree(os.path.join(ROOT, d), work / d, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = work / "oracle" / fname
    text = src.read_text()
    assert old in text, "mutation site moved: update the mutant"
    src.write_text(text.replace(old, new))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pins],
        cwd=work,
        capture_output=True,
        text=True,
        timeout=600,
        env=env,
    )
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
