"""Pins of the oracle's sub-grid, assembly and geometry (Sec. 4.1, 4.4)."""
import numpy as np
import pytest

from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from oracle.quadrature import tet_rule
from oracle.refelem import ref_element
from oracle.scheme import Oracle, dof_counts
from oracle.subgrid import build_cells, polyhedron_volume


def silvester(bary_w, N, lam, dlam):
    """Lagrange function of the lattice node with integer barycentric weights
    bary_w, phi = prod_i prod_{j<a_i} (N lam_i - j)/(j+1), and its gradient."""
    val = np.ones(lam.shape[0])
    grad = np.zeros((lam.shape[0], 3))
    factors = []
    for i in range(4):
        for j in range(bary_w[i]):
            factors.append(((N * lam[:, i] - j) / (j + 1), N * dlam[i] / (j + 1)))
    for f, _ in factors:
        val = val * f
    for a, (fa, da) in enumerate(factors):
        prod = np.ones(lam.shape[0])
        for b, (fb, _) in enumerate(factors):
            if b != a:
                prod = prod * fb
        grad += prod[:, None] * da[None, :]
    return val, grad


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_dof_count_formula_and_volumes(mesh_3, N):
    gs = build_cells(mesh_3, N)
    cnt = dof_counts(mesh_3, N)
    for c, g in gs.items():
        assert g.ndof == cnt[c] == len(set(g.keys))
        assert np.all(g.detJ > 0)
        assert abs(g.volume - polyhedron_volume(g)) < 1e-14
        assert np.abs((g.tri_area[:, None] * g.tri_normal).sum(0)).max() < 1e-15
    assert abs(sum(g.volume for g in gs.values()) - 1.0) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_mass_sum_is_cell_volume(mesh_3, N):
    """sum_{m,l} (M_i)_{ml} = |P_i| (partition of unity), volume by the divergence theorem."""
    o = Oracle(mesh_3, N)
    for c in range(mesh_3["n_cells"] if N < 4 else 6):  # P4: a sample, for time
        assert abs(o.mass(c).sum() - polyhedron_volume(o.grids[c])) < 1e-14


@pytest.mark.parametrize("N", [1, 2])
def test_face_pairing_is_geometric(mesh_3, N):
    """Paired face nodes are the same physical point (up to the periodic shift)."""
    gs = build_cells(mesh_3, N)
    L = mesh_3["box"]
    for c, g in gs.items():
        for k in range(len(g.conn)):
            h = gs[int(g.nbr[k])]
            xi = g.dof_x[g.face_dof[k]]
            xo = h.dof_x[g.nbr_face_dof[k]]
            d = xi - xo
            d -= L * np.round(d / L)
            assert np.abs(d).max() < 1e-13
            assert np.abs(g.tri_normal[k] + h.tri_normal[int(g.nbr_tri[k])]).max() == 0.0
            assert g.tri_area[k] == h.tri_area[int(g.nbr_tri[k])]


def _cube_mesh():
    """A 3^3 periodic lattice without jitter: every cell is a cube."""
    return periodic_voronoi(jittered_lattice_seeds(3, 0.0, 0))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("which", ["cube", "voronoi"])
def test_matrices_by_brute_force_quadrature(mesh_3, N, which):
    """Quadrature-free M_i and sum_k |J_k| sum_d G_k[d, x] K^_d against
    Grundmann-Moeller quadrature of the Lagrange functions evaluated from
    physical barycentric coordinates (4x4 solve per sub-tet)."""
    mesh = _cube_mesh() if which == "cube" else mesh_3
    o = Oracle(mesh, N)
    R = ref_element(N)
    bw = R.barycentric_weights()
    pts, wts = tet_rule(2 * N + 1)
    lam_ref = np.column_stack([1 - pts.sum(1), pts])
    for c in (0, 7) if N < 4 else (7,):  # P4: one cell, for time
        g = o.grids[c]
        M = np.zeros((g.ndof, g.ndof))
        S = np.zeros((3, g.ndof, g.ndof))
        for k in range(len(g.conn)):
            X = g.X[k]
            T = np.vstack([X.T, np.ones(4)])
            Tinv = np.linalg.inv(T)
            dlam = Tinv[:, :3]  # grad lambda_j = rows of T^{-1} (first 3 columns)
            vol = abs(np.linalg.det(T)) / 6.0
            phis, grads = [], []
            for m in range(R.np):
                v, gr = silvester(bw[m], N, lam_ref, dlam)
                phis.append(v)
                grads.append(gr)
            phis = np.array(phis)
            grads = np.array(grads)
            w = 6.0 * vol * wts
            idx = g.conn[k]
            M[np.ix_(idx, idx)] += np.einsum("q,mq,lq->ml", w, phis, phis)
            for x in range(3):
                S[x][np.ix_(idx, idx)] += np.einsum("q,mq,lq->ml", w, phis, grads[:, :, x])
        Mo = o.mass(c)
        assert np.abs(M - Mo).max() <= 1e-13 * np.abs(Mo).max()
        for x in range(3):
            So = np.zeros_like(Mo)
            for k in range(len(g.conn)):
                idx = g.conn[k]
                So[np.ix_(idx, idx)] += g.detJ[k] * np.einsum("d,dml->ml", g.G[k][:, x], R.K_f)
            assert np.abs(S[x] - So).max() <= 1e-12 * np.abs(So).max()


def test_complete_linkage_collapse_keeps_sub_tets_oriented():
    """Collapsing Voronoi edges shorter than 2% of the seed spacing by single
    linkage can chain many vertices of nearly co-spherical seeds into one
    point and invert sub-tetrahedra (7^3 jittered seeds, seed 38: one cell);
    complete linkage with the cluster at its mean keeps every cell's
    sub-tets of one orientation, and the cells still tile the box."""
    seeds = jittered_lattice_seeds(7, 0.25, 38)

    def inverted(mesh):
        gs = build_cells(mesh, 1)
        return sum(int(not (np.all(np.linalg.det(g.J) > 0) or np.all(np.linalg.det(g.J) < 0))) for g in gs.values()), gs

    bad, _ = inverted(periodic_voronoi(seeds, merge_tol=0.02 / 7))
    assert bad > 0
    bad, gs = inverted(periodic_voronoi(seeds, merge_tol=0.02 / 7, linkage="complete"))
    assert bad == 0
    assert abs(sum(polyhedron_volume(g) for g in gs.values()) - 1.0) < 1e-12
