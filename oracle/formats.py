"""Sparse storage formats beside CSR -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  The paper stores its matrices in CSR
and lists coordinate (COO), ELLPACK (ELL) and hybrid (HYB) storage as the
alternatives (Section 3.2, citing Saad's book and Bell and Garland); SELL-C-sigma
(Kreutzer et al., 2014) is the sliced ELL form for wide SIMD units.  Each
format is written out here from its definition, 0-based, complex128 values:

* ELL of width K: entry k of row i at position k*n + i (column-major, so that
  consecutive rows are consecutive in memory); a row's entries keep their CSR
  order in slots 0..len_i-1, slots len_i..K-1 are padding with column -1 and
  value 0.
* HYB of width K: the ELL part holds the first min(len_i, K) entries of each
  row, the COO part the rest as (row, column, value) triplets in CSR order.
  The default width is the largest K such that at least a third of the rows
  have K or more entries (Bell and Garland's rule).
* SELL-C-sigma with t lanes per row: rows are sorted by decreasing length
  within windows of sigma consecutive rows (ties keep their order; sigma = 1
  keeps the CSR order); sorted position p holds row perm[p] and belongs to
  chunk c = p // C as its row r = p % C; chunk c has width w_c = the
  longest row in it rounded up to a multiple of t and starts at chunk_ptr[c]
  (chunk_ptr[c+1] - chunk_ptr[c] = C w_c); entry k of that row sits at
  chunk_ptr[c] + (k // t) C t + r t + (k % t).  The last chunk is padded
  with empty rows; padding has column -1 and value 0.  t = 1 is the format
  of Kreutzer et al.; t > 1 splits each row over t neighbouring slots (the
  padded SELL-P layout of Anzt, Tomov and Dongarra).

Products skip padding and sum each row's entries in CSR order (for HYB: the
ELL part's sum plus the COO part's sum), so they equal the CSR product's
row sums entry for entry.
"""

from __future__ import annotations

import numpy as np

from workloads.csr import CSR


def row_lengths(A: CSR) -> np.ndarray:
    return np.diff(A.row_ptr).astype(np.int64)


def hyb_default_width(A: CSR) -> int:
    """Largest K with #{i : len_i >= K} >= ceil(n / 3) (0 for n = 0)."""
    n = A.n
    if n == 0:
        return 0
    lens = row_lengths(A)
    need = -(-n // 3)
    K = 0
    for k in range(1, int(lens.max()) + 1):
        if np.count_nonzero(lens >= k) >= need:
            K = k
    return K


def to_ell(A: CSR, K: int | None = None):
    """ELL(K) part and COO remainder.  Returns (K, col[K*n], val[K*n], coo_row, coo_col, coo_val)."""
    n = A.n
    lens = row_lengths(A)
    if K is None:
        K = int(lens.max()) if n else 0
    col = np.full(K * n, -1, dtype=np.int32)
    val = np.zeros(K * n, dtype=np.complex128)
    cr, cc, cv = [], [], []
    for i in range(n):
        lo, hi = int(A.row_ptr[i]), int(A.row_ptr[i + 1])
        for k in range(hi - lo):
            if k < K:
                col[k * n + i] = A.col_idx[lo + k]
                val[k * n + i] = A.vals[lo + k]
            else:
                cr.append(i)
                cc.append(A.col_idx[lo + k])
                cv.append(A.vals[lo + k])
    return (K, col, val, np.array(cr, dtype=np.int32), np.array(cc, dtype=np.int32),
            np.array(cv, dtype=np.complex128))


def ell_spmv(n, K, col, val, coo_row, coo_col, coo_val, x):
    """y_i = (sum over row i's ELL slots in order) + (sum over its COO entries in order)."""
    y = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        acc = 0j
        for k in range(K):
            c = col[k * n + i]
            if c >= 0:
                acc += val[k * n + i] * x[c]
        y[i] = acc
    extra = np.zeros(n, dtype=np.complex128)
    for r, c, v in zip(coo_row, coo_col, coo_val):
        extra[r] += v * x[c]
    has = np.zeros(n, dtype=bool)
    has[coo_row] = True
    y[has] += extra[has]
    return y


def ell_to_csr(n, K, col, val, coo_row, coo_col, coo_val) -> CSR:
    rows = [[] for _ in range(n)]
    for i in range(n):
        for k in range(K):
            if col[k * n + i] >= 0:
                rows[i].append((int(col[k * n + i]), val[k * n + i]))
    for r, c, v in zip(coo_row, coo_col, coo_val):
        rows[int(r)].append((int(c), v))
    return _csr_from_rows(rows)


def sell_perm(A: CSR, sigma: int) -> np.ndarray:
    """Sorted position -> row: decreasing length within windows of sigma rows, ties in row order."""
    n = A.n
    lens = row_lengths(A)
    perm = np.arange(n, dtype=np.int32)
    if sigma > 1:
        for w0 in range(0, n, sigma):
            rows = list(range(w0, min(n, w0 + sigma)))
            rows.sort(key=lambda i: -lens[i])  # Python's sort is stable
            perm[w0:w0 + len(rows)] = rows
    return perm


def to_sell(A: CSR, C: int, sigma: int, t: int = 1):
    """SELL-C-sigma with t lanes per row.  Returns (perm, chunk_ptr, col, val)."""
    n = A.n
    lens = row_lengths(A)
    perm = sell_perm(A, sigma)
    nch = -(-n // C)
    chunk_ptr = np.zeros(nch + 1, dtype=np.int64)
    for c in range(nch):
        rows = perm[c * C:(c + 1) * C]
        longest = int(lens[rows].max()) if len(rows) else 0
        w = -(-longest // t) * t
        chunk_ptr[c + 1] = chunk_ptr[c] + C * w
    col = np.full(int(chunk_ptr[-1]), -1, dtype=np.int32)
    val = np.zeros(int(chunk_ptr[-1]), dtype=np.complex128)
    for p in range(n):
        c, r = divmod(p, C)
        i = int(perm[p])
        lo = int(A.row_ptr[i])
        for k in range(int(lens[i])):
            q = int(chunk_ptr[c]) + (k // t) * C * t + r * t + (k % t)
            col[q] = A.col_idx[lo + k]
            val[q] = A.vals[lo + k]
    return perm, chunk_ptr, col, val


def sell_spmv(n, C, t, perm, chunk_ptr, col, val, x):
    y = np.zeros(n, dtype=np.complex128)
    for p in range(n):
        c, r = divmod(p, C)
        w = int(chunk_ptr[c + 1] - chunk_ptr[c]) // C
        acc = 0j
        for k in range(w):
            q = int(chunk_ptr[c]) + (k // t) * C * t + r * t + (k % t)
            if col[q] >= 0:
                acc += val[q] * x[col[q]]
        y[perm[p]] = acc
    return y


def sell_to_csr(n, C, t, perm, chunk_ptr, col, val) -> CSR:
    rows = [[] for _ in range(n)]
    for p in range(n):
        c, r = divmod(p, C)
        w = int(chunk_ptr[c + 1] - chunk_ptr[c]) // C
        for k in range(w):
            q = int(chunk_ptr[c]) + (k // t) * C * t + r * t + (k % t)
            if col[q] >= 0:
                rows[int(perm[p])].append((int(col[q]), val[q]))
    return _csr_from_rows(rows)


def _csr_from_rows(rows) -> CSR:
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c, _ in r], dtype=np.int32)
    v = np.array([x for r in rows for _, x in r], dtype=np.complex128)
    return CSR(rp, ci, v)
