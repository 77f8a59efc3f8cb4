"""Level-set (Cuthill-McKee) ordering and symmetric permutation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module.  The paper keeps matrices in the
order they come (CSR storage, Section 3.2); renumbering the unknowns is a
locality step of the GPU library, and BiCGStab with Jacobi scaling gives the
same iterates up to rounding for P A P^T (P x) = P b.  What the renumbering
produces has a plain definition, written out here:

* levels: the graph distance from a start node along the edges
  i -> col_idx[p] of the rows (-1 where unreached), by a queue-based
  breadth-first search in pure Python;
* start: a first search from node 0; the smallest index on its deepest level
  starts the second search (one step of the pseudo-peripheral node search);
* order (Cuthill-McKee): level 0 is the start; level L + 1 follows level L,
  its nodes sorted by the smallest new position of a neighbour on level L,
  then by degree (row length), then by index; unreached nodes last, in index
  order.  For a connected pattern this is the textbook Cuthill-McKee order
  (visit nodes in order, appending each one's unvisited neighbours by
  increasing degree) with ties broken by index.
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


def level_order(row_ptr, col_idx, bfs=None):
    """(perm, inv, level): perm[k] = old index of new row k (Cuthill-McKee); inv its inverse.

    ``bfs(row_ptr, col_idx, start) -> levels`` replaces the pure-Python search
    (for large patterns; any routine returning graph distances will do).
    """
    bfs = bfs or bfs_levels
    n = len(row_ptr) - 1
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    first = bfs(rp, ci, 0)
    deepest = int(first.max())
    start = int(np.flatnonzero(first == deepest)[0])
    level = bfs(rp, ci, start)
    deg = np.diff(rp)
    rows = np.repeat(np.arange(n), deg)
    # edges from a node on level L >= 1 to a neighbour on level L - 1, grouped by L
    up = (level[rows] >= 1) & (level[ci] == level[rows] - 1)
    er, ec = rows[up], ci[up]
    by = np.argsort(level[er], kind="stable")
    er, ec = er[by], ec[by]
    bounds = np.searchsorted(level[er], np.arange(int(level.max()) + 2))
    pos = np.full(n, -1, dtype=np.int64)
    pos[start] = 0
    order = [np.array([start])]
    cur = 1
    none = n  # no neighbour one level up (possible for a non-symmetric pattern): after the others
    for L in range(1, int(level.max()) + 1):
        nodes = np.flatnonzero(level == L)
        pmin = np.full(n, none, dtype=np.int64)
        lo, hi = bounds[L], bounds[L + 1]
        np.minimum.at(pmin, er[lo:hi], pos[ec[lo:hi]])
        srt = nodes[np.lexsort((nodes, deg[nodes], pmin[nodes]))]
        pos[srt] = cur + np.arange(len(srt))
        cur += len(srt)
        order.append(srt)
    order.append(np.flatnonzero(level < 0))
    perm = np.concatenate(order)
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
