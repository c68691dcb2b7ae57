"""The C ABI library on the CPU: it loads, exports every declared symbol, and
its host-only sub-grid construction matches the oracle bit-exactly."""
import re

import numpy as np
import pytest

from paper_2605_00619_amd import afe


def declared_symbols():
    src = open(__file__.replace("tests/test_library_host.py", "include/afe.h")).read()
    return sorted(set(re.findall(r"^(?:afe_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = afe.load()
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(afe.EXPORTED)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_host_subgrid_matches_oracle(mesh_4, N):
    from oracle.scheme import dof_counts
    from oracle.subgrid import build_cells
    h = afe.subgrid_host(mesh_4, N)
    gs = build_cells(mesh_4, N)
    n = mesh_4["n_cells"]
    assert np.array_equal(h["dof_ptr"], np.concatenate([[0], np.cumsum(dof_counts(mesh_4, N))]))
    assert np.array_equal(h["conn"], np.concatenate([gs[c].conn for c in range(n)]))
    sp = h["subtet_ptr"]
    assert np.array_equal(h["nbr_subtet"], np.concatenate([sp[gs[c].nbr] + gs[c].nbr_tri for c in range(n)]))
    assert np.array_equal(h["nbr_perm"], np.concatenate([gs[c].nbr_perm for c in range(n)]))
    G = np.concatenate([gs[c].G.reshape(-1, 9) for c in range(n)])
    dj = np.concatenate([gs[c].detJ for c in range(n)])
    assert np.abs(G - h["geo"][:, :9]).max() <= 1e-13 * np.abs(G).max()
    assert (np.abs(dj - h["geo"][:, 9]) / dj).max() < 1e-13
    a2 = np.concatenate([2 * gs[c].tri_area for c in range(n)])
    assert (np.abs(a2 - h["tri"][:, 0]) / a2).max() < 1e-14


@pytest.mark.parametrize("N", [1, 3])
def test_host_subgrid_matches_oracle_on_a_bounded_mesh(N):
    """Bounded mesh: the sub-grid equals the oracle's, boundary triangles are
    numbered in ascending sub-tet order with nbr_subtet = -1 - b and nbr_perm
    the identity."""
    from afe_inputs.mesh import box_voronoi, jittered_box_seeds
    from oracle.scheme import dof_counts
    from oracle.subgrid import build_cells
    L = (1.0, 1.2, 0.9)
    mesh = box_voronoi(jittered_box_seeds((3, 3, 3), L, 0.25, 4), L)
    h = afe.subgrid_host(mesh, N)
    gs = build_cells(mesh, N)
    n = mesh["n_cells"]
    assert np.array_equal(h["dof_ptr"], np.concatenate([[0], np.cumsum(dof_counts(mesh, N))]))
    assert np.array_equal(h["conn"], np.concatenate([gs[c].conn for c in range(n)]))
    sp = h["subtet_ptr"]
    onbr = np.concatenate([gs[c].nbr for c in range(n)])
    bnd = onbr < 0
    expect = np.concatenate([np.where(gs[c].nbr >= 0, sp[np.maximum(gs[c].nbr, 0)] + gs[c].nbr_tri, -1) for c in range(n)])
    expect[bnd] = -1 - np.arange(bnd.sum())
    assert np.array_equal(h["nbr_subtet"], expect)
    assert np.array_equal(h["nbr_perm"], np.concatenate([gs[c].nbr_perm for c in range(n)]))
    assert bnd.sum() > 0


def test_bad_mesh_and_budget_rejected(mesh_4):
    bad = dict(mesh_4)
    fc = mesh_4["face_cell"].copy()
    fc[0, 1] = fc[0, 0]
    bad["face_cell"] = fc
    with pytest.raises(afe.AfeError) as e:
        afe.subgrid_host(bad, 1)
    assert e.value.name == "AFE_E_BAD_MESH"
    with pytest.raises(afe.AfeError) as e:
        afe.CellData(mesh_4, 2, afe.Params(hbm_budget=1024), stream=0)
    assert e.value.name == "AFE_E_HBM_BUDGET"
    with pytest.raises(afe.AfeError) as e:
        afe.subgrid_host(mesh_4, 5)
    assert e.value.name == "AFE_E_ARG"
