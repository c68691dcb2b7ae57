"""Pins of the oracle's heat conduction (Sec. 2: energy flux - kappa grad T,
T = p / (rho R), R = (gamma - 1) c_v; second viscous eigenvalue
gamma mu / (Pr rho) with Pr = mu gamma c_v / kappa)."""
import math

import numpy as np

from oracle.physics import flux, pressure, prim_to_cons, visc_eig
from oracle.scheme import Oracle, Params

GAMMA, CV = 1.4, 2.5


def test_heat_flux_is_minus_kappa_times_the_temperature_gradient():
    """On a state that is affine in x, the change of the energy flux that kappa
    makes equals -kappa dT/dx_i, with dT/dx_i from a central difference of
    T = p / (rho R) along each direction; nothing else in the flux changes."""
    rng = np.random.default_rng(5)
    R = (GAMMA - 1.0) * CV
    kappa = 0.3
    q0 = prim_to_cons(np.array([1.2, 0.3, -0.2, 0.1, 0.9]), GAMMA)
    grad = rng.normal(size=(3, 5)) * 0.1  # grad[i, v] = d q_v / d x_i

    def T(q):
        return pressure(q, GAMMA) / (q[0] * R)

    h = 1e-5
    dT = np.array([(T(q0 + h * grad[i]) - T(q0 - h * grad[i])) / (2 * h) for i in range(3)])
    with_k = flux(q0, GAMMA, 0.0, grad, kappa, CV)
    without = flux(q0, GAMMA, 0.0, grad, 0.0, CV)
    assert np.abs((with_k[:, 4] - without[:, 4]) - (-kappa * dT)).max() < 1e-9 * kappa
    assert np.array_equal(with_k[:, :4], without[:, :4])
    # with viscosity as well, the heat term adds on top of the viscous energy flux
    both = flux(q0, GAMMA, 0.01, grad, kappa, CV)
    visc = flux(q0, GAMMA, 0.01, grad, 0.0, CV)
    assert np.abs((both[:, 4] - visc[:, 4]) - (-kappa * dT)).max() < 1e-9 * kappa


def test_thermal_eigenvalue_from_the_prandtl_number():
    """max(4 mu / (3 rho), gamma mu / (Pr rho)) with Pr = mu gamma c_v / kappa,
    for kappa on either side of the viscous one, and 4 mu / (3 rho) at kappa = 0."""
    q = prim_to_cons(np.array([[1.3, 0.1, 0.2, 0.3, 1.0]]), GAMMA)
    rho = 1.3
    for mu, kappa in ((1e-3, 1e-4), (1e-3, 1e-2), (2e-3, 0.0)):
        lam = 4.0 * mu / (3.0 * rho)
        if kappa > 0:
            pr = mu * GAMMA * CV / kappa
            lam = max(lam, GAMMA * mu / (pr * rho))
        assert abs(float(visc_eig(q, mu, kappa, CV)[0]) - lam) <= 1e-15 * lam


def test_heat_conduction_conserves_total_energy(mesh_3):
    """A resting gas with a temperature wave at uniform pressure: with kappa > 0
    energy moves between cells, but the face fluxes cancel pairwise, so mass,
    momentum and total energy (column sums of the cell mass matrices times the
    state) are conserved to rounding, and the energy does change."""
    R = (GAMMA - 1.0) * CV
    kappa = 5e-4

    def field(x, t=0.0):
        T = 1.0 + 0.1 * np.sin(2 * math.pi * x[:, 0])
        w = np.zeros((len(x), 5))
        w[:, 0] = 1.0 / (R * T)
        w[:, 4] = 1.0
        return w

    o = Oracle(mesh_3, 2, Params(kappa=kappa, cv=CV, tol=1e-14, max_iter=600))
    u0 = o.initial_state(field)
    dt = o.cfl_dt(u0, 0.004)
    u1, rep = o.step(u0, dt)
    assert rep.converged and rep.positive

    def totals(u):
        return sum(o.mass(c).sum(axis=0) @ o.cell_state(u, c) for c in range(o.n_cells))

    t0, t1 = totals(u0), totals(u1)
    assert np.abs(t1 - t0).max() < 1e-13 * np.abs(t0).max()
    assert np.abs(u1[4] - u0[4]).max() > 1e3 * 1e-16 * np.abs(u0[4]).max()
