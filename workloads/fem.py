"""P1 tetrahedral finite elements for the Helmholtz equation on voxel domains.

The paper's matrices come from the finite element discretisation of
-Lap(u) - k^2 u = g in car-cabin and cylinder cavities (Sections 2 and 3).
Those meshes are not public, so this module synthesises meshes of the same
kind: a structured hexahedral grid of spacing h is masked to the domain (a
grid cube is kept when its centre lies inside), every kept cube is split
into the 6 Kuhn tetrahedra, and interior nodes are jittered.

For the 6 permutations (p0, p1, p2) of the axes, the Kuhn tetrahedron of
the cube with lower corner c is (c, c+e_p0, c+e_p0+e_p1, c+(1,1,1)).  All
cubes use the same split, so the mesh is conforming.  Along each
tetrahedron's vertex list every coordinate is non-decreasing, so each edge
(earlier vertex -> later vertex) points along one of the 7 non-zero 0/1
vectors; the matrix couplings of a node are therefore stored in 8 "slots"
(the diagonal plus 7 positive directions), and the full matrix is the
mirror image of those upper slots.  Summing element contributions into the
slots in element order and mirroring makes A = A^T hold bitwise.

The complex system matrix is A = K - k^2 M + i k B with
    K_ab = |T| grad(phi_a) . grad(phi_b)      (stiffness)
    M_ab = |T| (1 + delta_ab) / 20            (consistent mass)
    B_ab = |F| (1 + delta_ab) / 12            (Robin boundary mass)
the standard P1 element integrals.  B is assembled on the boundary faces
selected as Robin (impedance) faces; other boundary faces are natural
(Neumann).
"""

from __future__ import annotations

from itertools import permutations

import numpy as np

from .csr import CSR, csr_from_coo, permute_symmetric

PERMS = list(permutations(range(3)))  # lexicographic order
UNIT = np.eye(3, dtype=np.int64)


def _slot(delta: np.ndarray) -> np.ndarray:
    """Slot code 4*dx + 2*dy + dz of a 0/1 direction (0 is the diagonal)."""
    return delta[..., 0] * 4 + delta[..., 1] * 2 + delta[..., 2]


SLOT_DIR = np.array([[(s >> 2) & 1, (s >> 1) & 1, s & 1] for s in range(8)], dtype=np.int64)


def kuhn_mesh(keep: np.ndarray, h: float, origin=(0.0, 0.0, 0.0), rng=None, jitter: float = 0.1) -> dict:
    """Kuhn-tetrahedral mesh of the kept cubes of a structured grid.

    ``keep`` is a bool array (nx, ny, nz) of kept grid cubes.  Nodes are the
    vertices of kept cubes, numbered in natural order of their grid position
    (x slowest).  Nodes on no boundary face are displaced by independent
    U(-jitter*h, jitter*h) draws per coordinate (one (n, 3) draw for all
    nodes, applied to interior nodes only).
    """
    keep = np.asarray(keep, dtype=bool)
    nx, ny, nz = keep.shape
    used = np.zeros((nx + 1, ny + 1, nz + 1), dtype=bool)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                used[dx : dx + nx, dy : dy + ny, dz : dz + nz] |= keep
    gid = np.full(used.shape, -1, dtype=np.int64)
    n = int(used.sum())
    gid[used] = np.arange(n, dtype=np.int64)
    gridpos = np.argwhere(used).astype(np.int64)  # C order == id order

    # Boundary squares: faces between a kept and a non-kept cube.
    pad = np.zeros((nx + 2, ny + 2, nz + 2), dtype=bool)
    pad[1:-1, 1:-1, 1:-1] = keep
    sq_corner, sq_axis, sq_plane = [], [], []
    for a in range(3):
        lo = [slice(1, -1)] * 3
        hi = [slice(1, -1)] * 3
        lo[a] = slice(0, -1)
        hi[a] = slice(1, None)
        diff = pad[tuple(lo)] ^ pad[tuple(hi)]  # face between cells (m-1, m) along a
        f = np.argwhere(diff).astype(np.int64)  # coordinate along a is the plane index m
        sq_corner.append(f)
        sq_axis.append(np.full(f.shape[0], a, dtype=np.int64))
        sq_plane.append(f[:, a].copy())
    sq_corner = np.concatenate(sq_corner)
    sq_axis = np.concatenate(sq_axis)

    bnode = np.zeros(n, dtype=bool)
    for a in range(3):
        sel = sq_axis == a
        g = sq_corner[sel]
        u, v = [ax for ax in range(3) if ax != a]
        for du in (0, 1):
            for dv in (0, 1):
                q = g + du * UNIT[u] + dv * UNIT[v]
                bnode[gid[q[:, 0], q[:, 1], q[:, 2]]] = True

    coords = np.asarray(origin, dtype=np.float64) + h * gridpos.astype(np.float64)
    if rng is not None and jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=(n, 3))
        coords[~bnode] += d[~bnode]

    cubes = np.argwhere(keep).astype(np.int64)  # C order
    tets = np.empty((cubes.shape[0], 6, 4), dtype=np.int64)
    for t, p in enumerate(PERMS):
        verts = [cubes, cubes + UNIT[p[0]], cubes + UNIT[p[0]] + UNIT[p[1]], cubes + 1]
        for v, q in enumerate(verts):
            tets[:, t, v] = gid[q[:, 0], q[:, 1], q[:, 2]]
    tets = tets.reshape(-1, 4)
    return {
        "n": n,
        "h": float(h),
        "coords": coords,
        "gridpos": gridpos,
        "gid": gid,
        "tets": tets,
        "sq_corner": sq_corner,
        "sq_axis": sq_axis,
        "boundary_node": bnode,
        "n_cubes": int(cubes.shape[0]),
    }


def _square_triangles(mesh: dict, sel: np.ndarray) -> np.ndarray:
    """Split the selected boundary squares into the two Kuhn triangles.

    On every face the Kuhn split uses the diagonal from the lower corner g to
    g + e_u + e_v (u < v the in-plane axes): triangles (g, g+e_u, g+e_u+e_v)
    and (g, g+e_v, g+e_u+e_v), vertices listed with non-decreasing coordinates.
    """
    gid = mesh["gid"]
    tris = []
    g_all, a_all = mesh["sq_corner"][sel], mesh["sq_axis"][sel]
    for a in range(3):
        g = g_all[a_all == a]
        if g.shape[0] == 0:
            continue
        u, v = [ax for ax in range(3) if ax != a]
        for mid in (UNIT[u], UNIT[v]):
            q = [g, g + mid, g + UNIT[u] + UNIT[v]]
            tris.append(np.stack([gid[x[:, 0], x[:, 1], x[:, 2]] for x in q], axis=1))
    if not tris:
        return np.zeros((0, 3), dtype=np.int64)
    t = np.concatenate(tris)
    assert np.all(t >= 0)
    return t


def _tet_local(coords: np.ndarray, tets: np.ndarray):
    """Volumes and upper-triangle local stiffness of every tetrahedron."""
    X = coords[tets]  # (T, 4, 3)
    e1, e2, e3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    c1, c2, c3 = np.cross(e2, e3), np.cross(e3, e1), np.cross(e1, e2)
    det = np.einsum("ij,ij->i", e1, c1)
    vol = np.abs(det) / 6.0
    # Barycentric gradients: columns of the inverse edge matrix.
    g = np.stack([-(c1 + c2 + c3), c1, c2, c3], axis=1) / det[:, None, None]  # (T, 4, 3)
    return vol, g


def assemble_helmholtz_p1(mesh: dict, k: float, robin_sel: np.ndarray) -> dict:
    """Assemble K, M, B on the mesh's edge pattern and A = K - k^2 M + i k B.

    ``robin_sel`` is a bool mask over the mesh's boundary squares selecting
    the Robin faces.  Returns a dict with the CSR matrix ``A`` and the real
    arrays ``K``, ``M``, ``B`` aligned with ``A``'s entries, plus ``tris``
    (the Robin triangles) and ``upper_pos`` (CSR position of every upper
    slot entry, used to map per-slot quantities onto the matrix).
    """
    n = mesh["n"]
    coords, tets, gridpos = mesh["coords"], mesh["tets"], mesh["gridpos"]
    vol, g = _tet_local(coords, tets)
    if not np.all(vol > 0):
        raise ValueError("non-positive tetrahedron volume")

    pairs = [(a, b) for a in range(4) for b in range(a, 4)]
    keys = np.empty((tets.shape[0], len(pairs)), dtype=np.int64)
    kloc = np.empty((tets.shape[0], len(pairs)), dtype=np.float64)
    mloc = np.empty((tets.shape[0], len(pairs)), dtype=np.float64)
    for q, (a, b) in enumerate(pairs):
        delta = gridpos[tets[:, b]] - gridpos[tets[:, a]]
        keys[:, q] = tets[:, a] * 8 + _slot(delta)
        kloc[:, q] = vol * np.einsum("ij,ij->i", g[:, a], g[:, b])
        mloc[:, q] = vol * ((2.0 if a == b else 1.0) / 20.0)
    keys = keys.ravel()
    nslot = 8 * n
    present = np.bincount(keys, minlength=nslot) > 0
    Ks = np.bincount(keys, weights=kloc.ravel(), minlength=nslot)
    Ms = np.bincount(keys, weights=mloc.ravel(), minlength=nslot)
    del kloc, mloc

    tris = _square_triangles(mesh, robin_sel)
    Bs = np.zeros(nslot)
    if tris.shape[0]:
        Xf = coords[tris]
        area = 0.5 * np.linalg.norm(np.cross(Xf[:, 1] - Xf[:, 0], Xf[:, 2] - Xf[:, 0]), axis=1)
        fp = [(a, b) for a in range(3) for b in range(a, 3)]
        fkeys = np.empty((tris.shape[0], len(fp)), dtype=np.int64)
        floc = np.empty((tris.shape[0], len(fp)), dtype=np.float64)
        for q, (a, b) in enumerate(fp):
            delta = gridpos[tris[:, b]] - gridpos[tris[:, a]]
            fkeys[:, q] = tris[:, a] * 8 + _slot(delta)
            floc[:, q] = area * ((2.0 if a == b else 1.0) / 12.0)
        fkeys = fkeys.ravel()
        if not np.all(present[fkeys]):
            raise AssertionError("Robin face edge missing from the tetrahedral pattern")
        Bs = np.bincount(fkeys, weights=floc.ravel(), minlength=nslot)

    slots = np.flatnonzero(present)
    i = slots // 8
    s = slots % 8
    jpos = gridpos[i] + SLOT_DIR[s]
    j = mesh["gid"][jpos[:, 0], jpos[:, 1], jpos[:, 2]]
    assert np.all(j >= 0)
    off = s > 0
    rows = np.concatenate([i, j[off]])
    cols = np.concatenate([j, i[off]])
    src = np.concatenate([slots, slots[off]])  # slot feeding each entry
    A = csr_from_coo(n, rows, cols, np.zeros(rows.shape[0], dtype=np.complex128))
    # csr_from_coo sorted by (row, col); recover the permutation it applied.
    key = rows.astype(np.int64) * n + cols
    order = np.argsort(key, kind="stable")
    src_sorted = src[order]
    K, M, B = Ks[src_sorted], Ms[src_sorted], Bs[src_sorted]
    A.vals = (K - (k * k) * M) + 1j * (k * B)
    upper_pos = np.empty(nslot, dtype=np.int64)
    upper_pos[:] = -1
    inv = np.empty_like(order)
    inv[order] = np.arange(order.shape[0])
    upper_pos[slots] = inv[: slots.shape[0]]
    A.meta = {"kind": "p1", "n": n, "h": mesh["h"], "k": float(k)}
    return {"A": A, "K": K, "M": M, "B": B, "tris": tris, "upper_pos": upper_pos, "slot_of_entry": src_sorted}


def cylinder_mesh(
    h: float = 0.04, radius: float = 1.0, length: float = 4.0, rng=None, jitter: float = 0.1, robin: str = "all"
):
    """Cylinder along x: keep cubes whose centre has y^2 + z^2 <= radius^2.

    ``robin="caps"``: impedance only on the end caps x = 0 and x = length,
    the lateral staircase wall natural (Neumann).  ``robin="all"``
    (default): impedance on the caps and on the lateral wall.  The two give
    the same sparsity pattern; with caps only the system is a nearly
    undamped waveguide on which BiCGStab stagnates.
    """
    nx = int(round(length / h))
    ny = nz = int(round(2 * radius / h))
    yc = -radius + h * (np.arange(ny) + 0.5)
    zc = -radius + h * (np.arange(nz) + 0.5)
    disc = (yc[:, None] ** 2 + zc[None, :] ** 2) <= radius * radius
    keep = np.broadcast_to(disc, (nx, ny, nz)).copy()
    mesh = kuhn_mesh(keep, h, origin=(0.0, -radius, -radius), rng=rng, jitter=jitter)
    ax, g = mesh["sq_axis"], mesh["sq_corner"]
    caps = (ax == 0) & ((g[:, 0] == 0) | (g[:, 0] == nx))
    if robin == "caps":
        mesh["robin_sel"] = caps
    elif robin == "all":
        mesh["robin_sel"] = np.ones_like(caps)
    else:
        raise ValueError("robin must be 'caps' or 'all'")
    mesh["domain"] = {"shape": "cylinder", "radius": radius, "length": length, "grid": (nx, ny, nz)}
    return mesh


def cabin_mesh(h: float = 0.012, dims=(2.0, 1.2, 1.1), rng=None, jitter: float = 0.1, seat=(0.6, 0.5, 1.0)):
    """Box with two seat-shaped box cutouts standing on the floor.

    Draw order from ``rng``: the two seat x-offsets ~ U(0.3, 1.1), then the
    two seat y-offsets ~ U(0, 0.05) added to 0.05 (left) and 0.65 (right),
    then the node jitter.  Robin faces are all outer box faces; the seat
    surfaces are natural (Neumann).
    """
    if rng is None:
        raise ValueError("cabin_mesh needs an rng for the seat placement")
    nx, ny, nz = (int(round(d / h)) for d in dims)
    x0 = rng.uniform(0.3, 1.1, size=2)
    y0 = np.array([0.05, 0.65]) + rng.uniform(0.0, 0.05, size=2)
    xc = h * (np.arange(nx) + 0.5)
    yc = h * (np.arange(ny) + 0.5)
    zc = h * (np.arange(nz) + 0.5)
    X, Y, Z = np.meshgrid(xc, yc, zc, indexing="ij")
    keep = np.ones((nx, ny, nz), dtype=bool)
    for s in range(2):
        inside = (
            (X >= x0[s]) & (X <= x0[s] + seat[0]) & (Y >= y0[s]) & (Y <= y0[s] + seat[1]) & (Z >= 0.0) & (Z <= seat[2])
        )
        keep &= ~inside
    del X, Y, Z
    mesh = kuhn_mesh(keep, h, rng=rng, jitter=jitter)
    ax, g = mesh["sq_axis"], mesh["sq_corner"]
    plane = g[np.arange(g.shape[0]), ax]
    ext = np.array([nx, ny, nz])[ax]
    mesh["robin_sel"] = (plane == 0) | (plane == ext)
    mesh["domain"] = {
        "shape": "cabin",
        "dims": (nx * h, ny * h, nz * h),
        "grid": (nx, ny, nz),
        "seats_x0": x0.tolist(),
        "seats_y0": y0.tolist(),
    }
    return mesh


def permute_problem(A: CSR, perm: np.ndarray) -> CSR:
    return permute_symmetric(A, perm)
