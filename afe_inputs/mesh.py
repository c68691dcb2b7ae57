"""Seeded Voronoi meshes of a box: periodic ([0, L)^3) or bounded
([0, Lx] x [0, Ly] x [0, Lz], cells clipped to the box).

This module only generates input geometry: it knows nothing of the AFE
sub-grid, the basis or the scheme.  Both the CPU oracle and the HIP library
consume the arrays it returns, each building its own sub-grid from them.

Mesh arrays (all numpy, C order):
    xyz          float64 [nv, 3]   one canonical coordinate per vertex, in [0, L)
    face_ptr     int32   [nf + 1]  CSR offsets into face_vtx
    face_vtx     int32   [sum]     polygon corners, cyclic, oriented outward
                                   from the owner cell (right-hand rule)
    face_vshift  int8    [sum, 3]  image shift of each corner: its position in
                                   the owner's frame is xyz[v] + shift * L
    face_cell    int32   [nf, 2]   (owner, neighbour); neighbour -1 marks a face
                                   on the boundary of a bounded mesh
    nbr_shift    int8    [nf, 3]   neighbour seed in the owner's frame is
                                   seeds[nbr] + nbr_shift * L
    seeds        float64 [nc, 3]
    box          float64           L (bounded meshes: the largest side; no
                                   shifts are used there)
    bounded      bool              True for a bounded mesh (all shifts zero)
    lengths      float64 [3]       box sides (bounded meshes)
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Voronoi, cKDTree


def jittered_lattice_seeds(n: int, jitter: float, seed: int, box: float = 1.0) -> np.ndarray:
    """n^3 seeds: lattice points ((i, j, k) + 1/2) h, h = box/n, each moved by a
    uniform offset in [-jitter*h, +jitter*h]^3 and wrapped into the box.

    Lattice order is C order over (i, j, k) with i along x (k varies fastest);
    the jitter is drawn as one (n^3, 3) uniform array from default_rng(seed).
    """
    h = box / n
    idx = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter * h, jitter * h, size=(n ** 3, 3))
    pts = (idx + 0.5) * h + jit
    return np.mod(pts, box)


def uniform_seeds(m: int, seed: int, box: float = 1.0) -> np.ndarray:
    """m seeds drawn uniformly in the box (Poisson-Voronoi statistics)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, box, size=(m, 3))


def _images(seeds: np.ndarray, box: float, margin: float):
    """Seeds plus the periodic images that fall within `margin` of the box."""
    n = len(seeds)
    pts = [seeds]
    ids = [np.arange(n)]
    shifts = [np.zeros((n, 3), dtype=np.int64)]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                if sx == 0 and sy == 0 and sz == 0:
                    continue
                s = np.array([sx, sy, sz])
                p = seeds + s * box
                keep = np.all((p > -margin) & (p < box + margin), axis=1)
                pts.append(p[keep])
                ids.append(np.nonzero(keep)[0])
                shifts.append(np.tile(s, (int(keep.sum()), 1)))
    return np.concatenate(pts), np.concatenate(ids), np.concatenate(shifts)


def periodic_voronoi(seeds: np.ndarray, box: float = 1.0, margin: float | None = None,
                     merge_tol: float | None = None, linkage: str = "single") -> dict:
    """Periodic Voronoi tessellation of `seeds` in [0, box)^3.

    Every vertex is stored once (a single canonical coordinate in [0, box)),
    and each face once, owned by the lower cell id; corners carry integer image
    shifts so that both cells see bit-identical corner coordinates up to a
    translation by a multiple of `box`.

    Voronoi vertices closer than merge_tol * box are merged into one (periodic
    copies of one vertex, and the clusters that nearly co-spherical seeds
    produce); polygon corners that coincide after the merge are removed and
    polygons left with fewer than three corners vanish.  The default merges
    vertices closer than 1e-3 of the mean seed spacing box / n^(1/3): it turns
    Voronoi edges shorter than that into points, which removes the
    sub-tetrahedral slivers of relative volume down to 1e-10 that such edges
    create; merge_tol = 1e-10 keeps the exact diagram.

    linkage "single" merges every chain of vertices closer than the
    tolerance into one cluster placed at its lowest-numbered member;
    "complete" merges two clusters only while every pair of their members
    stays within the tolerance (closest pairs first) and places a cluster at
    the mean of its members, which keeps the cells star-shaped where long
    chains of nearly co-spherical seeds would invert sub-tetrahedra.
    """
    seeds = np.asarray(seeds, dtype=np.float64)
    n = len(seeds)
    if n < 27:
        raise ValueError("periodic Voronoi needs at least 27 seeds (no self-neighbour faces)")
    if margin is None:
        margin = 4.0 * box / n ** (1.0 / 3.0)
    if merge_tol is None:
        merge_tol = 1e-3 / n ** (1.0 / 3.0)
    pts, pid, psh = _images(seeds, box, margin)
    vor = Voronoi(pts)

    # canonical vertex table: wrap every Voronoi vertex used by an original
    # cell into [0, box) and merge copies that coincide up to merge_tol*box
    rp = vor.ridge_points
    own_mask = (rp[:, 0] < n) | (rp[:, 1] < n)
    used = sorted({v for r, m in zip(vor.ridge_vertices, own_mask) if m for v in r})
    if -1 in used:
        raise RuntimeError("unbounded Voronoi region touches an original cell; increase margin")
    used = np.array(used)
    vpos = vor.vertices[used]
    wrapped = np.mod(vpos, box)
    wrapped[wrapped >= box] -= box
    tree = cKDTree(wrapped, boxsize=box)
    pairs = tree.query_pairs(merge_tol * box, output_type="ndarray")
    parent = np.arange(len(used))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    if linkage not in ("single", "complete"):
        raise ValueError("linkage must be 'single' or 'complete'")
    members = {i: [i] for i in range(len(used))}
    if linkage == "complete" and len(pairs):
        dd = wrapped[pairs[:, 0]] - wrapped[pairs[:, 1]]
        dd -= box * np.round(dd / box)
        pairs = pairs[np.argsort(np.linalg.norm(dd, axis=1), kind="stable")]
    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra == rb:
            continue
        if linkage == "complete":
            d = wrapped[members[ra]][:, None, :] - wrapped[members[rb]][None, :, :]
            d -= box * np.round(d / box)
            if np.linalg.norm(d, axis=2).max() > merge_tol * box:
                continue
        lo, hi = min(ra, rb), max(ra, rb)
        parent[hi] = lo
        members[lo] = members[lo] + members.pop(hi)
    roots = np.array([find(i) for i in range(len(used))])
    uroots, canon = np.unique(roots, return_inverse=True)
    xyz = wrapped[uroots].copy()
    if linkage == "complete":
        for k, r in enumerate(uroots):
            if len(members[r]) > 1:
                d = wrapped[members[r]] - wrapped[r]
                d -= box * np.round(d / box)
                xyz[k] = np.mod(wrapped[r] + d.mean(axis=0), box)
    # a merged cluster must stay small next to the seed spacing (nearly
    # co-spherical seeds chain up to ~16 vertices of a 2% merge into one)
    spread = np.linalg.norm(wrapped - xyz[canon] - box * np.round((wrapped - xyz[canon]) / box), axis=1)
    if spread.max() > 0.1 * box / n ** (1.0 / 3.0):
        raise RuntimeError("merge tolerance too large for this seed spacing")
    vmap = -np.ones(len(vor.vertices), dtype=np.int64)
    vmap[used] = canon

    faces = {}
    for r, (a, b) in enumerate(rp):
        for own, oth in ((a, b), (b, a)):
            if own >= n:
                continue
            co, cn = int(pid[own]), int(pid[oth])
            s = psh[oth] - psh[own]
            if co == cn:
                raise RuntimeError("self-neighbour face; mesh too coarse")
            if co < cn:
                key = (co, cn, tuple(int(x) for x in s))
                if key not in faces:
                    faces[key] = r
    keys = sorted(faces)
    face_ptr = [0]
    face_vtx, face_vshift, face_cell, nbr_shift = [], [], [], []
    for key in keys:
        r = faces[key]
        a, b = rp[r]
        own = a if (a < n and pid[a] == key[0] and not psh[a].any()) else b
        oth = b if own == a else a
        po = pts[own]
        pn = pts[oth]
        nrm = pn - po
        nrm /= np.linalg.norm(nrm)
        vids = np.array(vor.ridge_vertices[r])
        # one corner per merged vertex
        _, first = np.unique(vmap[vids], return_index=True)
        vids = vids[np.sort(first)]
        if len(vids) < 3:
            continue
        vp = vor.vertices[vids]
        ctr = vp.mean(axis=0)
        e1 = vp[0] - ctr
        e1 -= nrm * np.dot(e1, nrm)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        ang = np.arctan2((vp - ctr) @ e2, (vp - ctr) @ e1)
        order = np.argsort(ang)
        vids, vp = vids[order], vp[order]
        # positions in the owner's frame: owner seed is an original point
        g = vmap[vids]
        sh = np.rint((vp - xyz[g]) / box).astype(np.int64)
        if np.abs(vp - (xyz[g] + sh * box)).max() > 0.1 * box / n ** (1.0 / 3.0):
            raise RuntimeError("vertex image shift mismatch")
        face_vtx.extend(g.tolist())
        face_vshift.extend(sh.tolist())
        face_ptr.append(len(face_vtx))
        face_cell.append((key[0], key[1]))
        nbr_shift.append(key[2])
    mesh = dict(
        xyz=np.ascontiguousarray(xyz, dtype=np.float64),
        face_ptr=np.array(face_ptr, dtype=np.int32),
        face_vtx=np.array(face_vtx, dtype=np.int32),
        face_vshift=np.array(face_vshift, dtype=np.int8).reshape(-1, 3),
        face_cell=np.array(face_cell, dtype=np.int32).reshape(-1, 2),
        nbr_shift=np.array(nbr_shift, dtype=np.int8).reshape(-1, 3),
        seeds=seeds.copy(),
        box=float(box),
        n_cells=n,
        bounded=False,
        lengths=np.full(3, float(box)),
    )
    _check_closed(mesh)
    return mesh


def jittered_box_seeds(counts, lengths, jitter: float, seed: int) -> np.ndarray:
    """nx ny nz seeds in [0, Lx] x [0, Ly] x [0, Lz]: lattice points
    ((i, j, k) + 1/2) h_d, h_d = L_d / n_d, each moved by a uniform offset in
    [-jitter h_d, +jitter h_d] per direction (jitter < 1/2 keeps every seed
    inside).  Lattice in C order over (i, j, k); the offsets are one
    (nx ny nz, 3) uniform draw of default_rng(seed), scaled per direction."""
    counts = np.asarray(counts, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.float64)
    if not 0.0 <= jitter < 0.5:
        raise ValueError("jitter must lie in [0, 1/2)")
    h = lengths / counts
    idx = np.stack(np.meshgrid(*(np.arange(c) for c in counts), indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=(len(idx), 3)) * h
    return (idx + 0.5) * h + jit


def box_voronoi(seeds: np.ndarray, lengths, merge_tol: float | None = None) -> dict:
    """Voronoi tessellation of `seeds` clipped to the box [0, Lx] x [0, Ly] x
    [0, Lz].

    The diagram is taken of the seeds together with their mirror images
    across the six box planes: for a point inside the box a mirror image is
    never nearer than the seed it mirrors, and outside the box beyond a plane
    the seed's own mirror is nearer than the seed, so each seed's cell is its
    Voronoi cell clipped to the box, and the face between a seed and its own
    mirror lies in the plane.  Faces to a mirror are boundary faces
    (neighbour -1).  Vertices closer than merge_tol times the mean seed
    spacing are merged as in periodic_voronoi (default 1e-3 of the mean
    spacing); every cell must stay inside the box and the cell volumes must
    add up to the box volume (checked by the callers' tests)."""
    seeds = np.asarray(seeds, dtype=np.float64)
    lengths = np.asarray(lengths, dtype=np.float64).reshape(3)
    n = len(seeds)
    if n < 2:
        raise ValueError("a bounded Voronoi mesh needs at least 2 seeds")
    if np.any(seeds <= 0.0) or np.any(seeds >= lengths):
        raise ValueError("seeds must lie inside the box")
    spacing = float(np.prod(lengths) / n) ** (1.0 / 3.0)
    if merge_tol is None:
        merge_tol = 1e-3
    margin = 4.0 * spacing
    pts, mir = [seeds], [np.arange(n)]
    for d in range(3):
        for side in (0.0, lengths[d]):
            near = np.abs(seeds[:, d] - side) < margin
            p = seeds[near].copy()
            p[:, d] = 2.0 * side - p[:, d]
            pts.append(p)
            mir.append(np.nonzero(near)[0])
    pts = np.concatenate(pts)
    orig = np.concatenate(mir)  # seed each point is (an image of)
    vor = Voronoi(pts)
    rp = vor.ridge_points
    own_mask = (rp[:, 0] < n) | (rp[:, 1] < n)
    used = sorted({v for r, m in zip(vor.ridge_vertices, own_mask) if m for v in r})
    if -1 in used:
        raise RuntimeError("unbounded Voronoi region touches a cell")
    used = np.array(used)
    vpos = vor.vertices[used]
    tol = 1e-9 * float(lengths.max())
    if np.any(vpos < -tol) or np.any(vpos > lengths + tol):
        raise RuntimeError("a cell reaches outside the box")
    vpos = np.clip(vpos, 0.0, lengths)
    tree = cKDTree(vpos)
    pairs = tree.query_pairs(merge_tol * spacing, output_type="ndarray")
    parent = np.arange(len(used))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(len(used))])
    uroots, canon = np.unique(roots, return_inverse=True)
    xyz = vpos[uroots].copy()
    if np.linalg.norm(vpos - xyz[canon], axis=1).max() > 0.1 * spacing:
        raise RuntimeError("merge tolerance too large for this seed spacing")
    # a merged vertex stays on every box plane one of its members lies on
    for d in range(3):
        for side in (0.0, lengths[d]):
            on = np.abs(vpos[:, d] - side) <= tol
            xyz[np.unique(canon[on]), d] = side
    vmap = -np.ones(len(vor.vertices), dtype=np.int64)
    vmap[used] = canon

    faces = []  # (owner, neighbour or -1, ridge)
    for r, (a, b) in enumerate(rp):
        if a >= n and b >= n:
            continue
        if a < n and b < n:
            faces.append((min(a, b), max(a, b), r))
        else:
            own, oth = (a, b) if a < n else (b, a)
            faces.append((int(own), -1, r))
    faces.sort()
    face_ptr = [0]
    face_vtx, face_cell = [], []
    for own, nb, r in faces:
        a, b = rp[r]
        oth = b if a == own else a
        nrm = pts[oth] - pts[own]
        nrm /= np.linalg.norm(nrm)
        vids = np.array(vor.ridge_vertices[r])
        _, first = np.unique(vmap[vids], return_index=True)
        vids = vids[np.sort(first)]
        if len(vids) < 3:
            continue
        vp = vor.vertices[vids]
        ctr = vp.mean(axis=0)
        e1 = vp[0] - ctr
        e1 -= nrm * np.dot(e1, nrm)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        order = np.argsort(np.arctan2((vp - ctr) @ e2, (vp - ctr) @ e1))
        face_vtx.extend(vmap[vids[order]].tolist())
        face_ptr.append(len(face_vtx))
        face_cell.append((own, nb))
    nfc = len(face_cell)
    mesh = dict(
        xyz=np.ascontiguousarray(xyz, dtype=np.float64),
        face_ptr=np.array(face_ptr, dtype=np.int32),
        face_vtx=np.array(face_vtx, dtype=np.int32),
        face_vshift=np.zeros((len(face_vtx), 3), dtype=np.int8),
        face_cell=np.array(face_cell, dtype=np.int32).reshape(-1, 2),
        nbr_shift=np.zeros((nfc, 3), dtype=np.int8),
        seeds=seeds.copy(),
        box=float(lengths.max()),
        n_cells=n,
        bounded=True,
        lengths=lengths.copy(),
    )
    _check_closed(mesh)
    return mesh


def _check_closed(mesh: dict) -> None:
    """Every cell must see each of its vertices at one single image shift and
    every edge of a cell's boundary must be used by exactly two of its faces."""
    n = mesh["n_cells"]
    fp, fv, fs = mesh["face_ptr"], mesh["face_vtx"], mesh["face_vshift"].astype(np.int64)
    fc, ns = mesh["face_cell"], mesh["nbr_shift"].astype(np.int64)
    vshift = [dict() for _ in range(n)]
    edges = [dict() for _ in range(n)]
    for f in range(len(fc)):
        for side in (0, 1):
            c = int(fc[f, side])
            if c < 0:
                continue
            corners = list(range(fp[f], fp[f + 1]))
            if side == 1:
                corners = corners[::-1]
            for k, ci in enumerate(corners):
                v = int(fv[ci])
                s = tuple(fs[ci] - (ns[f] if side == 1 else 0))
                if vshift[c].setdefault(v, s) != s:
                    raise RuntimeError(f"cell {c} sees vertex {v} at two images")
                w = int(fv[corners[(k + 1) % len(corners)]])
                edges[c][(v, w)] = edges[c].get((v, w), 0) + 1
    for c in range(n):
        for (v, w), cnt in edges[c].items():
            if cnt != 1 or edges[c].get((w, v), 0) != 1:
                raise RuntimeError(f"cell {c} is not a closed oriented surface")


def mesh_stats(mesh: dict) -> dict:
    """Counts used to size buffers: faces per cell, polygon edges per cell."""
    n = mesh["n_cells"]
    fp, fc = mesh["face_ptr"], mesh["face_cell"]
    nf = np.zeros(n, dtype=np.int64)
    ne2 = np.zeros(n, dtype=np.int64)
    for f in range(len(fc)):
        k = fp[f + 1] - fp[f]
        for c in fc[f]:
            if c < 0:
                continue
            nf[c] += 1
            ne2[c] += k
    return dict(faces_per_cell=nf, subtets_per_cell=ne2)
