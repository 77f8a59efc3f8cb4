"""A plain container for a square complex CSR matrix (paper Section 3.2).

The paper stores a sparse matrix as three arrays: values ``AA``, column
indices ``JA`` and row starts ``IA`` (1-based, ``IA(n+1) = nz + 1``).  Here
the same three arrays are 0-based: row ``i`` occupies
``[row_ptr[i], row_ptr[i+1])`` of ``col_idx`` / ``vals``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray  # complex128 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def check(self) -> None:
        """Structural checks only (no arithmetic of the method)."""
        rp, ci = self.row_ptr, self.col_idx
        assert rp.dtype == np.int32 and ci.dtype == np.int32
        assert rp[0] == 0 and rp[-1] == ci.shape[0] == self.vals.shape[0]
        assert np.all(np.diff(rp) >= 0)
        assert ci.size == 0 or (ci.min() >= 0 and ci.max() < self.n)

    def with_vals(self, vals: np.ndarray) -> "CSR":
        return CSR(self.row_ptr, self.col_idx, np.ascontiguousarray(vals), dict(self.meta))

    def row_of_entry(self) -> np.ndarray:
        """Row index of every stored entry (int64 [nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def stats(self) -> dict:
        """Matrix statistics in the sense of the paper's matrix table (Section 3.1).

        ``density`` is in percent, ``bandwidth`` is the upper bandwidth
        max(j - i), ``max_row`` the longest row and ``mean``/``stddev`` the
        row-length mean and standard deviation.
        """
        lens = np.diff(self.row_ptr).astype(np.float64)
        rows = self.row_of_entry()
        band = int(np.max(self.col_idx.astype(np.int64) - rows)) if self.nnz else 0
        return {
            "n": self.n,
            "nnz": self.nnz,
            "density_pct": 100.0 * self.nnz / float(self.n) ** 2,
            "bandwidth": band,
            "max_row": int(lens.max()),
            "mean_row": float(lens.mean()),
            "stddev_row": float(lens.std()),
        }


def csr_from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sort entries by (row, col) and compress.  Entries must be unique."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) entries")
    r = rows[order]
    counts = np.bincount(r, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(
        row_ptr.astype(np.int32),
        np.ascontiguousarray(cols[order].astype(np.int32)),
        np.ascontiguousarray(vals[order].astype(np.complex128)),
    )


def permute_symmetric(A: CSR, perm: np.ndarray) -> CSR:
    """Return P A P^T where node ``i`` is renumbered ``perm[i]``."""
    rows = perm[A.row_of_entry()]
    cols = perm[A.col_idx.astype(np.int64)]
    out = csr_from_coo(A.n, rows, cols, A.vals)
    out.meta = dict(A.meta)
    return out
