"""Bounded meshes and the Dirichlet boundary data of the oracle (reading R21
in oracle/scheme.py; Sec. 5.1-5.2 impose the exact solution on all sides).

- The bounded Voronoi mesh (afe_inputs.mesh.box_voronoi): the cell volumes,
  computed here by the divergence theorem from the face polygons, add up to
  the box volume; every boundary face lies in one of the six box planes; the
  boundary faces of a jittered lattice are one per lattice cell on each side.
- An affine translating density (rho = rho0 + g . (x - v t), constant v and
  p) is an exact Euler solution inside the space-time polynomial space of
  every degree N >= 1, and every flux is affine in rho: the predictor
  reproduces it, interior faces see equal states, and a boundary triangle
  given the exact solution at the right positions and time nodes sees equal
  states too.  So one step from t must give the exact nodal values at t + dt
  to round-off; a boundary datum taken at a wrong time, place or weight
  breaks this at the size of the translation over the step.
- A uniform flow with its own value as boundary data is preserved.
- With viscosity: the linear shear v = (0, a (x - x0), 0) at rho = 1 heated
  uniformly by its own dissipation (p = p0 + (gamma - 1) mu a^2 t) is an
  exact Navier-Stokes solution whose state and fluxes lie in the P3
  space-time space (the kinetic-energy flux is cubic in x), so one N = 3 step
  with the exact state and gradient as boundary data reproduces it to
  round-off, also with heat conduction on (the temperature is uniform).
"""
import numpy as np
import pytest

from afe_inputs.fields import affine_density, shear_heating, shear_heating_grad, uniform_state
from afe_inputs.mesh import box_voronoi, jittered_box_seeds
from oracle.physics import prim_to_cons
from oracle.scheme import Oracle, Params


def _box_mesh(n=3, L=(1.0, 1.2, 0.9), seed=4):
    return box_voronoi(jittered_box_seeds((n, n, n), L, 0.25, seed), L)


def _cell_volumes(mesh):
    fp, fv, xyz, fc = mesh["face_ptr"], mesh["face_vtx"], mesh["xyz"], mesh["face_cell"]
    vol = np.zeros(mesh["n_cells"])
    for f in range(len(fc)):
        P = xyz[fv[fp[f]:fp[f + 1]]]
        c0 = P.mean(0)
        v = sum(np.dot(c0, np.cross(P[i], P[(i + 1) % len(P)])) for i in range(len(P))) / 6.0
        vol[fc[f, 0]] += v
        if fc[f, 1] >= 0:
            vol[fc[f, 1]] -= v
    return vol


@pytest.mark.parametrize("merge_tol", [None, 0.05])
def test_box_mesh_fills_the_box(merge_tol):
    """Also with short edges collapsed: merged vertices keep the box planes
    of their members, so the boundary stays on the box."""
    L = np.array([1.0, 1.2, 0.9])
    m = box_voronoi(jittered_box_seeds((4, 4, 4), L, 0.25, 4), L, merge_tol=merge_tol)
    vol = _cell_volumes(m)
    assert vol.min() > 0.0
    assert abs(vol.sum() - L.prod()) < 1e-12 * L.prod()
    fp, fv, xyz, fc = m["face_ptr"], m["face_vtx"], m["xyz"], m["face_cell"]
    bnd = np.nonzero(fc[:, 1] < 0)[0]
    assert len(bnd) == 6 * 4 * 4
    for f in bnd:
        P = xyz[fv[fp[f]:fp[f + 1]]]
        on = [(d, s) for d in range(3) for s in (0.0, L[d]) if np.abs(P[:, d] - s).max() < 1e-12]
        assert len(on) == 1, P


@pytest.mark.parametrize("N", [1, 2])
def test_affine_solution_reproduced_with_boundary_data(N):
    mesh = _box_mesh()
    t0 = 0.3
    exact = lambda x, t: affine_density(x, t, grad=(0.3, 0.2, 0.25), vel=(0.8, 0.5, 0.6))
    o = Oracle(mesh, N, Params(tol=1e-14, max_iter=300), boundary=exact)
    u = o.initial_state(lambda x: exact(x, t0))
    dt = 10.0 * o.cfl_dt(u, 0.01)  # one step; the affine fixed point is reached at any dt
    un, rep = o.step(u, dt, t=t0)
    assert rep.converged and rep.positive
    ref = prim_to_cons(exact(o.dof_coords().T, t0 + dt), 1.4).T
    err = np.abs(un - ref).max() / np.abs(ref).max()
    moved = np.abs(u - ref).max() / np.abs(ref).max()
    assert moved > 1e-4  # the state changes by far more than the bar
    print(f"N={N}: moved {moved:.2e}, error {err:.2e}")
    assert err < 1e-13, (err, moved)


def test_uniform_flow_preserved_with_boundary_data():
    mesh = _box_mesh()
    flow = lambda x, t=0.0: uniform_state(x)
    o = Oracle(mesh, 2, Params(tol=1e-14, max_iter=300), boundary=flow)
    u = o.initial_state(flow)
    dt = o.cfl_dt(u, 0.02)
    un, rep = o.step(u, dt, t=0.0)
    assert rep.converged
    assert np.abs(un - u).max() < 1e-13 * np.abs(u).max()


@pytest.mark.parametrize("kappa", [0.0, 0.02])
def test_viscous_shear_reproduced_with_boundary_data(kappa):
    """On the 3^3 box mesh with short edges collapsed, at the workloads' CFL
    number 0.004: error 1.4e-12 against a change of 1.2e-6 over the step (the
    viscous predictor's stop at 1e-14 leaves that much, as for the
    artificial-viscosity parity cases); a boundary datum at the wrong time or
    without its gradient is off by the size of the change."""
    mu = 0.05
    exact = lambda x, t: shear_heating(x, t, a=0.8, mu=mu)
    grad = lambda x, t: shear_heating_grad(x, t, a=0.8)
    L = (1.0, 1.2, 0.9)
    mesh = box_voronoi(jittered_box_seeds((3, 3, 3), L, 0.25, 4), L, merge_tol=0.02)
    o = Oracle(mesh, 3, Params(mu=mu, kappa=kappa, tol=1e-14, max_iter=600), boundary=exact, boundary_grad=grad)
    t0 = 0.2
    u = o.initial_state(lambda x: exact(x, t0))
    dt = o.cfl_dt(u, 0.004)
    un, rep = o.step(u, dt, t=t0)
    assert rep.converged and rep.positive
    ref = prim_to_cons(exact(o.dof_coords().T, t0 + dt), 1.4).T
    err = np.abs(un - ref).max() / np.abs(ref).max()
    moved = np.abs(u - ref).max() / np.abs(ref).max()
    print(f"kappa={kappa}: moved {moved:.2e}, error {err:.2e}")
    assert moved > 1e-6 and err < 1e-11, (err, moved)


def test_viscous_boundary_needs_the_gradient():
    o = Oracle(_box_mesh(), 1, Params(mu=0.01), boundary=lambda x, t: uniform_state(x))
    u = o.initial_state(uniform_state)
    with pytest.raises(ValueError):
        o.step(u, 1e-4)
