"""Pins of the oracle's Navier-Stokes terms, its Rusanov face flux and its face
mass matrix, each against a value fixed outside the oracle:

- the Stokes stress of Sec. 2 on affine velocity fields, where the stress
  tensor and the viscous energy flux have closed forms worked out by hand
  (simple shear, uniform dilatation with zero bulk viscosity, shear under a
  density gradient);
- the time-integrated Rusanov flux with viscous penalty of Sec. 4.4
  (eq. 3.33) on a face between two constant states at rest, whose value is
  written out from the states' numbers;
- the face mass matrix Z^ (Sec. 4.4) entry by entry against a quadrature of
  the basis products on the face t = 0 of the reference tetrahedron;
- the kinetic-energy dissipation rate of the Taylor-Green vortex at t = 0,
  dE_k/dt = -mu int |grad v|^2 = -(3/4) mu (2 pi)^3 for the classical field on
  [0, 2 pi]^3 (a property of the continuous equations of Sec. 2), against one
  oracle step with and without viscosity;
- the predictor's fixed point (eq:ader4) against a direct dense solve where
  the map is affine: on the density wave (constant velocity and pressure)
  every flux is affine in the density.
"""
import math

import numpy as np
import pytest

from afe_inputs.fields import density_wave, taylor_green_3d
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from oracle.physics import flux, prim_to_cons
from oracle.quadrature import tet_rule, tri_rule
from oracle.refelem import ref_element
from oracle.scheme import Oracle, Params

GAMMA = 1.4


def _state_and_gradient(rho, grad_rho, vel, grad_vel, p, grad_p):
    """Conserved state q and its gradient dq_v/dx_i at one point from the
    primitive values and their gradients (grad_vel[i, j] = d v_j / d x_i),
    by the product rule, written out per variable."""
    rho_v = rho * vel
    E = p / (GAMMA - 1.0) + 0.5 * rho * vel @ vel
    q = np.array([rho, *rho_v, E])
    g = np.zeros((3, 5))
    for i in range(3):
        g[i, 0] = grad_rho[i]
        g[i, 1:4] = grad_rho[i] * vel + rho * grad_vel[i]
        g[i, 4] = grad_p[i] / (GAMMA - 1.0) + 0.5 * grad_rho[i] * vel @ vel + rho * vel @ grad_vel[i]
    return q, g


def test_stress_simple_shear():
    """v = (a y, 0, 0), rho = 1.3, p = 0.8 at y = 0.4 with a = 0.5, mu = 0.02:
    div v = 0, the only velocity derivative is dv_x/dy = a, so
    sigma = p I - mu a (e_x e_y + e_y e_x): sigma_xy = sigma_yx = -0.01,
    sigma_xx = sigma_yy = sigma_zz = 0.8.  Momentum flux rho v_i v_j + sigma_ij
    with v = (0.2, 0, 0); energy flux v_i (rho E) + sigma_ij v_j."""
    a, mu, y, rho, p = 0.5, 0.02, 0.4, 1.3, 0.8
    vel = np.array([a * y, 0.0, 0.0])
    gv = np.zeros((3, 3))
    gv[1, 0] = a
    q, g = _state_and_gradient(rho, np.zeros(3), vel, gv, p, np.zeros(3))
    F = flux(q, GAMMA, mu, g)
    rhoE = p / 0.4 + 0.5 * rho * 0.04  # 2.026
    expect = np.zeros((3, 5))
    expect[0] = [rho * 0.2, rho * 0.04 + 0.8, -0.01, 0.0, 0.2 * rhoE + 0.8 * 0.2]
    expect[1] = [0.0, -0.01, 0.8, 0.0, -0.01 * 0.2]
    expect[2] = [0.0, 0.0, 0.0, 0.8, 0.0]
    assert np.abs(F - expect).max() < 1e-15


def test_stress_uniform_dilatation():
    """v = a x (uniform expansion), a = 0.3, mu = 0.05: div v = 3a and
    grad v = a I, so the Stokes hypothesis (zero bulk viscosity) leaves no
    viscous normal stress: sigma = (p + 2 mu a - 2 mu a) I = p I."""
    a, mu, rho, p = 0.3, 0.05, 0.9, 1.1
    x = np.array([0.2, -0.1, 0.3])
    vel = a * x
    q, g = _state_and_gradient(rho, np.zeros(3), vel, a * np.eye(3), p, np.zeros(3))
    Fv = flux(q, GAMMA, mu, g)
    Fi = flux(q, GAMMA, 0.0, None)
    assert np.abs(Fv - Fi).max() < 1e-15
    # the inviscid flux itself: rho v_i v_j + p delta_ij, v_i (rho E + p)
    rhoE = q[4]
    assert np.abs(Fi[:, 1:4] - (rho * np.outer(vel, vel) + p * np.eye(3))).max() < 1e-15
    assert np.abs(Fi[:, 4] - vel * (rhoE + p)).max() < 1e-15


def test_stress_under_a_density_gradient_and_compression():
    """v = (-b x, a x, 0) with a = 0.4, b = 0.25 at x = (0.5, 0, 0), mu = 0.1,
    rho = 2 + 3 x, p = 1 + x: the velocity gradient is recovered from the
    conserved gradient whatever the density gradient; dv_x/dx = -b,
    dv_y/dx = a, div v = -b, so
        sigma_xx = p + (2/3) mu (-b) - 2 mu (-b) = p + (4/3) mu b
        sigma_yy = sigma_zz = p - (2/3) mu b
        sigma_xy = sigma_yx = -mu a
    with p = 1.5: 1.5333..., 1.48333..., -0.04."""
    a, b, mu = 0.4, 0.25, 0.1
    X = 0.5
    rho, p = 2.0 + 3.0 * X, 1.0 + X
    vel = np.array([-b * X, a * X, 0.0])
    gv = np.zeros((3, 3))
    gv[0, 0] = -b
    gv[0, 1] = a
    q, g = _state_and_gradient(rho, np.array([3.0, 0, 0]), vel, gv, p, np.array([1.0, 0, 0]))
    F = flux(q, GAMMA, mu, g)
    sxx, syy, sxy = 1.5 + 4.0 / 3.0 * 0.025, 1.5 - 2.0 / 3.0 * 0.025, -0.04
    sigma = np.array([[sxx, sxy, 0.0], [sxy, syy, 0.0], [0.0, 0.0, syy]])
    assert np.abs(F[:, 1:4] - (rho * np.outer(vel, vel) + sigma)).max() < 1e-14
    assert np.abs(F[:, 4] - (vel * q[4] + sigma @ vel)).max() < 1e-14


def _constant_traces(o, c, q, dt):
    """Time-integrated traces of a constant state at rest on every boundary
    triangle of cell c: qbar = dt q, Fbar = dt F with F = p I in the momentum
    rows and zero mass and energy flux (v = 0)."""
    g = o.grids[c]
    K, nf = len(g.conn), len(o.ref.face_nodes_a)
    p = (GAMMA - 1.0) * q[4]
    F = np.zeros((3, 5))
    for i in range(3):
        F[i, 1 + i] = p
    return dict(tq=np.broadcast_to(dt * q, (K, nf, 5)).copy(), tF=np.broadcast_to(dt * F, (K, nf, 3, 5)).copy())


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_rusanov_flux_two_states_at_rest(mesh_3, N):
    """Eq. 3.33 on a face between this cell (rho = 1) and its neighbour
    (rho = 4), both at rest with p = 1/gamma, so c = 1 and 0.5.  With the cell
    viscosities 0.03 and 0.06 the viscous eigenvalues 4 mu / (3 rho) are 0.04
    and 0.02.  Per unit time: G = (1/2)(F+ + F-).n - (1/2) s (q+ - q-),
    s = max(|v.n| + c) + 2 eps max lambda^v = 1 + 2 eps 0.04,
    eps = (2N+1) / ((h+ + h-) sqrt(pi/2)); q+ - q- = (3, 0, 0, 0, 0) and the
    averaged flux is p n in the momentum rows."""
    o = Oracle(mesh_3, N)
    c, k, dt = 4, 2, 0.01
    g = o.grids[c]
    nb = int(g.nbr[k])
    p = 1.0 / GAMMA
    qm = np.array([1.0, 0.0, 0.0, 0.0, p / (GAMMA - 1.0)])
    qp = np.array([4.0, 0.0, 0.0, 0.0, p / (GAMMA - 1.0)])
    ti = {c: _constant_traces(o, c, qm, dt), nb: _constant_traces(o, nb, qp, dt)}
    mus = {c: 0.03, nb: 0.06}
    G = o.rusanov(c, k, ti, mus, dt)
    n = g.tri_normal[k]
    eps = (2 * N + 1) / ((g.h + o.grids[nb].h) * math.sqrt(math.pi / 2.0))
    s = 1.0 + 2.0 * eps * 0.04
    expect = np.array([-0.5 * s * 3.0, p * n[0], p * n[1], p * n[2], 0.0]) * dt
    assert np.abs(G - expect[None, :]).max() < 1e-15
    # the penalty is the viscous one: without viscosity s = 1 exactly
    G0 = o.rusanov(c, k, ti, {c: 0.0, nb: 0.0}, dt)
    assert np.abs(G0[:, 0] + 1.5 * dt).max() < 1e-15


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_face_mass_entrywise(N):
    """Z^[i][j] = int over the reference triangle (t = 0, area 1/2) of
    phi_{fn_i} phi_{fn_j}, by a Grundmann-Moeller rule exact to degree 2N+1;
    the basis functions of nodes off the face vanish on it."""
    R = ref_element(N)
    tp, tw = tri_rule(2 * N + 1)
    x = np.column_stack([tp, np.zeros(len(tp))])
    phi = R.eval_basis(x)
    Zq = np.einsum("q,qi,qj->ij", tw, phi, phi)
    fn = R.face_nodes_a
    # the Grundmann-Moeller rule's own rounding (mixed-sign weights) is 2e-15 at degree 9
    assert np.abs(R.Z_f - Zq[np.ix_(fn, fn)]).max() < 1e-14
    off = np.setdiff1d(np.arange(R.np), fn)
    assert np.abs(phi[:, off]).max() < 1e-13


def _kinetic_energy(o, u):
    """int rho |v|^2 / 2 over the target cells, each sub-tet by a
    Grundmann-Moeller rule of degree 2N + 3 (the paper's norms integrate the
    same way)."""
    pts, wts = tet_rule(2 * o.N + 3)
    phi = o.ref.eval_basis(pts)
    tot = 0.0
    for c in o.targets:
        g = o.grids[c]
        uc = o.cell_state(u, c)
        for k in range(len(g.conn)):
            q = phi @ uc[g.conn[k]]
            tot += g.detJ[k] * float(wts @ (0.5 * (q[:, 1:4] ** 2).sum(1) / q[:, 0]))
    return tot


def test_taylor_green_dissipation_rate():
    """Classical 3D Taylor-Green field on [0, 2 pi]^3 (rho = 1, Mach 0.1): at
    t = 0 it is divergence free and dE_k/dt = -mu int |grad v|^2
    = -(3/4) mu (2 pi)^3.  One oracle step (3^3 seeds, N = 2) with mu = 0.01
    and one without viscosity from the same state and time step: the
    difference of the kinetic energies is the viscous dissipation over the
    step.  Measured ratio to -(3/4) mu (2 pi)^3 dt: 0.9995.  A stress without
    the transposed gradient would double it."""
    box = 2 * math.pi
    mesh = periodic_voronoi(jittered_lattice_seeds(3, 0.25, 3, box=box), box=box)
    mu = 0.01
    field = lambda x: taylor_green_3d(x, mach=0.1)
    o0 = Oracle(mesh, 2, Params(tol=1e-14, max_iter=600))
    u0 = o0.initial_state(field)
    dt = o0.cfl_dt(u0, 0.004)
    ue, rep0 = o0.step(u0, dt)
    om = Oracle(mesh, 2, Params(mu=mu, tol=1e-14, max_iter=600))
    uv, rep1 = om.step(u0, dt)
    assert rep0.converged and rep1.converged
    ratio = (_kinetic_energy(om, uv) - _kinetic_energy(o0, ue)) / (-0.75 * mu * box ** 3 * dt)
    assert abs(ratio - 1.0) < 0.02, ratio


@pytest.mark.parametrize("N", [1, 2])
def test_predictor_fixed_point_equals_direct_solve(mesh_3, N):
    """On the density wave (velocity (1,1,1), p = 1) every flux is affine in
    rho, so on states of that form eq:ader4 is an affine map of the
    space-time density values, r -> b + T r.  Its matrix is read column by
    column from the map itself; the accelerated iteration's fixed point must
    equal the dense solution of (I - T) r = b."""
    o = Oracle(mesh_3, N, Params(tol=1e-14, max_iter=600))
    u = o.initial_state(density_wave)
    dt = o.cfl_dt(u, 0.004)
    c = 7
    un = o.cell_state(u, c)
    A, n = N + 1, o.grids[c].ndof
    vel = np.ones(3)

    def lift(r):  # [A, n] densities -> [A, n, 5] conserved states
        q = np.empty((A, n, 5))
        q[..., 0] = r
        q[..., 1:4] = r[..., None] * vel
        q[..., 4] = 1.0 / (GAMMA - 1.0) + 0.5 * r * 3.0
        return q

    r0 = np.ones((A, n))
    g0 = o.predictor_map(c, lift(r0), un, dt, 0.0)[..., 0]
    T = np.empty((A * n, A * n))
    for j in range(A * n):
        e = np.zeros(A * n)
        e[j] = 1.0
        T[:, j] = (o.predictor_map(c, lift(r0 + e.reshape(A, n)), un, dt, 0.0)[..., 0] - g0).ravel()
    b = g0.ravel() - T @ r0.ravel()
    r_direct = np.linalg.solve(np.eye(A * n) - T, b)
    q, it, ok = o.predictor(c, un, dt, 0.0)
    assert ok
    assert np.abs(q[..., 0].ravel() - r_direct).max() < 1e-12
    # the iterate stays on the affine family: momentum = rho (1,1,1), p = 1
    assert np.abs(q[..., 1:4] - q[..., :1] * vel).max() < 1e-12
