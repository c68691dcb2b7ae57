"""Sub-tetrahedral grid of each polyhedral cell and its agglomerated DOFs.

Sec. 4.1: each polyhedron P_i is split into sub-tetrahedra T_ik that cover it
conformingly; on each the P_N Lagrange basis is used, and the cell DOFs are
the union "without repetition" of all sub-tet nodes, which makes the
representation continuous inside P_i and discontinuous across cells.

Split used here (the paper allows any conforming one): every polygon face is
fanned about its vertex-mean centroid F and each resulting triangle is coned
to the vertex-mean centroid C of the cell, giving the sub-tet (a, b, F, C) for
each polygon edge (a, b) taken in the face's outward cyclic order.  Each
sub-tet has exactly one face on the cell boundary, the triangle (a, b, F).

Reference map: x = X0 + J xi with J = [X1-X0 | X2-X0 | X3-X0] and
(X0, X1, X2, X3) = (a, b, F, C); |det J| = 6 vol (|T^| = 1/6).

DOF numbering (a convention; any fixed one gives the same discrete space):
a node is keyed by the sorted tuple of (sub-grid vertex id, integer
barycentric weight > 0); sub-grid vertex ids order mesh vertices by global id,
then face centroids by global face id, then the cell centroid.  DOFs are
numbered by ascending (entity dimension, key).
"""
from __future__ import annotations

import numpy as np

from .refelem import ref_element

# sub-grid vertex ids: (type, global id); type 0 mesh vertex, 1 face centroid, 2 cell centroid
_VTX, _FACE, _CELL = 0, 1, 2


class CellGrid:
    """Everything the scheme needs about one cell.

    ndof            number of cell DOFs N_i
    keys            [ndof] node keys, in DOF order
    dof_x           [ndof, 3] DOF coordinates in the cell's frame
    conn            [K, np] sub-tet node -> cell DOF
    X               [K, 4, 3] sub-tet vertices (a, b, F, C)
    J, detJ, G      [K, 3, 3] Jacobian, |det J| [K], G = J^{-1} (row d = grad xi_d)
    tri_area        [K] area of each sub-tet's boundary triangle
    tri_normal      [K, 3] unit normal of it, outward from this cell
    nbr             [K] neighbour cell across that triangle (-1: boundary of a
                    bounded mesh; then nbr_tri = -1, nbr_face_dof = -1)
    nbr_tri         [K] index of the same triangle among the neighbour's sub-tets
    nbr_perm        [K, nf] face node j of this triangle is node nbr_perm[j] of the neighbour's
    face_dof        [K, nf] cell DOF of each face node
    nbr_face_dof    [K, nf] neighbour's cell DOF of each face node
    h               cell diameter (largest vertex distance)
    vertices        [V, 3] polyhedron vertices in the cell's frame
    faces           list of (global face id, corner coordinates [k, 3] outward)
    """


def _cell_faces(mesh: dict, c: int, cell_faces: list[list[tuple[int, int]]]):
    """Faces of cell c in its own frame, oriented outward: list of
    (face id, corner vertex ids, corner coordinates)."""
    L = mesh["box"]
    fp, fv = mesh["face_ptr"], mesh["face_vtx"]
    fs = mesh["face_vshift"].astype(np.float64)
    ns = mesh["nbr_shift"].astype(np.float64)
    xyz = mesh["xyz"]
    out = []
    for f, side in cell_faces[c]:
        idx = np.arange(fp[f], fp[f + 1])
        shift = fs[idx] if side == 0 else fs[idx] - ns[f]
        pos = xyz[fv[idx]] + shift * L
        vids = fv[idx]
        if side == 1:
            pos = pos[::-1]
            vids = vids[::-1]
        out.append((f, np.array(vids), pos))
    return out


def faces_of_cells(mesh: dict) -> list[list[tuple[int, int]]]:
    """For each cell the list of (face id, side) with side 0 = owner, 1 = neighbour."""
    n = mesh["n_cells"]
    lst = [[] for _ in range(n)]
    for f, (o, nb) in enumerate(mesh["face_cell"]):
        lst[int(o)].append((f, 0))
        if nb >= 0:  # a bounded mesh's boundary faces have no neighbour
            lst[int(nb)].append((f, 1))
    return lst


def _face_geometry_owner(mesh: dict, f: int):
    """Owner-frame corners and centroid of face f (oriented outward from owner)."""
    L = mesh["box"]
    fp, fv = mesh["face_ptr"], mesh["face_vtx"]
    idx = np.arange(fp[f], fp[f + 1])
    pos = mesh["xyz"][fv[idx]] + mesh["face_vshift"][idx].astype(np.float64) * L
    return fv[idx], pos, pos.mean(axis=0)


def build_cell(mesh: dict, c: int, N: int, cell_faces=None) -> CellGrid:
    """Sub-grid of one cell; neighbour pairing is filled by build_cells."""
    R = ref_element(N)
    bw = R.barycentric_weights()
    if cell_faces is None:
        cell_faces = faces_of_cells(mesh)
    faces = _cell_faces(mesh, c, cell_faces)
    # cell vertices in this cell's frame
    vpos = {}
    for f, vids, pos in faces:
        for v, p in zip(vids, pos):
            v = int(v)
            if v in vpos and not np.array_equal(vpos[v], p):
                raise ValueError(f"cell {c}: vertex {v} at two positions")
            vpos[v] = p
    vid_sorted = sorted(vpos)
    verts = np.array([vpos[v] for v in vid_sorted])
    C = verts.mean(axis=0)
    subtets = []  # (ids(4), coords(4,3), face id)
    for f, vids, pos in faces:
        F = pos.mean(axis=0)
        k = len(vids)
        for e in range(k):
            a, b = e, (e + 1) % k
            ids = ((_VTX, int(vids[a])), (_VTX, int(vids[b])), (_FACE, int(f)), (_CELL, 0))
            subtets.append((ids, np.array([pos[a], pos[b], F, C]), f))
    K = len(subtets)
    npn = R.np
    node_keys = []
    for ids, X, f in subtets:
        row = []
        for m in range(npn):
            key = tuple(sorted((ids[j], int(bw[m, j])) for j in range(4) if bw[m, j] > 0))
            row.append(key)
        node_keys.append(row)
    uniq = sorted({k for row in node_keys for k in row}, key=lambda k: (len(k) - 1, k))
    dof_of = {k: i for i, k in enumerate(uniq)}
    g = CellGrid()
    g.cell = c
    g.N = N
    g.ndof = len(uniq)
    g.keys = uniq
    g.dof_of = dof_of
    g.conn = np.array([[dof_of[k] for k in row] for row in node_keys], dtype=np.int64)
    g.face_dof = g.conn[:, R.face_nodes_a]
    g.X = np.stack([X for _, X, _ in subtets])
    g.sub_ids = [ids for ids, _, _ in subtets]
    g.sub_face = np.array([f for _, _, f in subtets], dtype=np.int64)
    g.tri_index = {(int(f), ids[0][1], ids[1][1]): k for k, (ids, _, f) in enumerate(subtets)}
    g.J = np.stack([np.column_stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]]) for X in g.X])
    g.detJ = np.abs(np.linalg.det(g.J))
    g.G = np.linalg.inv(g.J)
    # DOF coordinates: reference node mapped through its sub-tet
    dx = np.zeros((g.ndof, 3))
    for k in range(K):
        dx[g.conn[k]] = g.X[k, 0] + R.nodes_f @ g.J[k].T
    g.dof_x = dx
    g.vertices = verts
    g.faces = [(f, pos) for f, _, pos in faces]
    d = verts[:, None, :] - verts[None, :, :]
    g.h = float(np.sqrt((d * d).sum(-1)).max())
    g.volume = float(g.detJ.sum() / 6.0)
    return g


def build_cells(mesh: dict, N: int, cells=None) -> dict[int, CellGrid]:
    """Sub-grids of the requested cells (default: all) and of their
    neighbours, with boundary triangles paired across every face.

    Boundary-triangle area and normal are computed once per face in the owner's
    frame and negated for the neighbour, so both sides use identical values.
    """
    n = mesh["n_cells"]
    cf = faces_of_cells(mesh)
    if cells is None:
        cells = range(n)
    cells = sorted(set(int(c) for c in cells))
    need = set(cells)
    for c in cells:
        for f, side in cf[c]:
            other = int(mesh["face_cell"][f][1 - side])
            if other >= 0:
                need.add(other)
    grids = {c: build_cell(mesh, c, N, cf) for c in sorted(need)}
    R = ref_element(N)
    fn = R.face_nodes_a
    # owner-frame triangle geometry per (face, directed edge)
    tri_geo = {}
    for c in cells:
        g = grids[c]
        K = len(g.conn)
        g.tri_area = np.zeros(K)
        g.tri_normal = np.zeros((K, 3))
        g.nbr = np.zeros(K, dtype=np.int64)
        g.nbr_tri = np.zeros(K, dtype=np.int64)
        g.nbr_perm = np.zeros((K, len(fn)), dtype=np.int64)
        g.nbr_face_dof = np.zeros((K, len(fn)), dtype=np.int64)
        for k in range(K):
            f = int(g.sub_face[k])
            o, nb = (int(x) for x in mesh["face_cell"][f])
            a_id, b_id = g.sub_ids[k][0][1], g.sub_ids[k][1][1]
            if f not in tri_geo:
                vids, pos, F = _face_geometry_owner(mesh, f)
                geo = {}
                kk = len(vids)
                for e in range(kk):
                    a, b = pos[e], pos[(e + 1) % kk]
                    cr = np.cross(b - a, F - a)
                    nrm = np.linalg.norm(cr)
                    geo[(int(vids[e]), int(vids[(e + 1) % kk]))] = (0.5 * nrm, cr / nrm)
                tri_geo[f] = geo
            if c == o:
                area, nvec = tri_geo[f][(a_id, b_id)]
                other = nb
            else:
                area, nvec = tri_geo[f][(b_id, a_id)]
                nvec = -nvec
                other = o
            g.tri_area[k] = area
            g.tri_normal[k] = nvec
            g.nbr[k] = other
            if other < 0:  # boundary triangle of a bounded mesh: no partner
                g.nbr_tri[k] = -1
                g.nbr_perm[k] = np.arange(len(fn))
                g.nbr_face_dof[k] = -1
                continue
            h = grids[other]
            # neighbour's sub-tet on the same triangle: edge (b, a) on face f
            kn = h.tri_index[(f, b_id, a_id)]
            g.nbr_tri[k] = kn
            my_keys = [g.keys[g.conn[k, m]] for m in fn]
            nb_keys = [h.keys[h.conn[kn, m]] for m in fn]
            pos_in_nb = {key: j for j, key in enumerate(nb_keys)}
            g.nbr_perm[k] = [pos_in_nb[key] for key in my_keys]
            g.nbr_face_dof[k] = [h.dof_of[key] for key in my_keys]
    return grids


def polyhedron_volume(g: CellGrid) -> float:
    """Volume enclosed by the cell's boundary surface by the divergence theorem:
    each polygon (possibly non-planar) is the fan of triangles (a, b, F) about
    its vertex-mean centroid F, and |P| = 1/6 sum det[a, b, F] over all fan
    triangles (signed tetrahedra with the origin)."""
    tot = 0.0
    for _, pos in g.faces:
        k = len(pos)
        F = pos.mean(axis=0)
        for e in range(k):
            tot += float(np.linalg.det(np.array([pos[e], pos[(e + 1) % k], F]))) / 6.0
    return tot
