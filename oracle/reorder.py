"""Level-set ordering and symmetric permutation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module.  The paper keeps matrices in the
order they come (CSR storage, Section 3.2); renumbering the unknowns is a
locality step of the GPU library, and BiCGStab with Jacobi scaling gives the
same iterates up to rounding for P A P^T (P x) = P b.  What the renumbering
produces has a plain definition, written out here with a queue-based
breadth-first search in pure Python:

* levels: the graph distance from a start node along the edges
  i -> col_idx[p] of the rows (-1 where unreached);
* start: a first search from node 0; the smallest index on its deepest level
  starts the second search (one step of the pseudo-peripheral node search);
* order: nodes sorted by (level of the second search, index), unreached
  nodes last in index order.

Pure Python loops: meant for the small and medium patterns of the tests.
"""

from __future__ import annotations

from collections import deque

import numpy as np


def bfs_levels(row_ptr, col_idx, start: int) -> np.ndarray:
    """Graph distance of every node from ``start`` (-1 if unreachable)."""
    n = len(row_ptr) - 1
    rp = [int(v) for v in row_ptr]
    ci = [int(v) for v in col_idx]
    level = [-1] * n
    level[start] = 0
    q = deque([start])
    while q:
        i = q.popleft()
        li = level[i] + 1
        for p in range(rp[i], rp[i + 1]):
            j = ci[p]
            if level[j] < 0:
                level[j] = li
                q.append(j)
    return np.asarray(level, dtype=np.int64)


def level_order(row_ptr, col_idx):
    """(perm, inv, level): perm[k] = old index of new row k; inv its inverse."""
    n = len(row_ptr) - 1
    first = bfs_levels(row_ptr, col_idx, 0)
    deepest = int(first.max())
    start = int(np.flatnonzero(first == deepest)[0])
    level = bfs_levels(row_ptr, col_idx, start)
    key = np.where(level < 0, int(level.max()) + 1, level)
    perm = np.lexsort((np.arange(n), key))
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    return perm, inv, level


def permute(row_ptr, col_idx, vals, perm, inv):
    """P A P^T in CSR: row k is old row perm[k], columns renumbered by inv and sorted."""
    n = len(row_ptr) - 1
    rp = np.zeros(n + 1, dtype=np.int64)
    cis, vs = [], []
    for k in range(n):
        o = int(perm[k])
        lo, hi = int(row_ptr[o]), int(row_ptr[o + 1])
        c = np.asarray(inv)[np.asarray(col_idx[lo:hi], dtype=np.int64)]
        order = np.argsort(c, kind="stable")
        cis.append(c[order])
        vs.append(np.asarray(vals[lo:hi])[order])
        rp[k + 1] = rp[k] + (hi - lo)
    ci = np.concatenate(cis) if cis else np.zeros(0, dtype=np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, dtype=np.complex128)
    return rp, ci, v
