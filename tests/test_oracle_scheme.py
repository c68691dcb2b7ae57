"""Pins of the oracle's step: closed-form predictor solutions, invariants of
the scheme, and the formulas of the detector and the time step."""
import math

import numpy as np
import pytest

from afe_inputs.fields import density_wave, uniform_state
from oracle.physics import cons_to_prim, prim_to_cons
from oracle.scheme import Oracle, Params


def _affine_field(coef):
    """rho = 1 + coef . x, u = (1, 1, 1) translated in time, p = 1."""
    vel = np.ones(3)

    def f(x, t=0.0):
        w = np.zeros((len(x), 5))
        w[:, 0] = 1.0 + (x - vel * t) @ coef
        w[:, 1:4] = vel
        w[:, 4] = 1.0
        return w
    return f


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_predictor_reproduces_translated_polynomial(mesh_3, N):
    """A field whose exact solution lies in the space-time polynomial space is
    reproduced by the local space-time Galerkin predictor (Sec. 4.3): with
    rho = 1 + c.(x - u t), u, p constant, every flux is polynomial of degree
    <= N in x and 1 in t, so the fixed point is the exact translation."""
    o = Oracle(mesh_3, N, Params(depth=8, tol=1e-12))
    coef = np.array([0.3, -0.2, 0.25])
    f = _affine_field(coef)
    c = 5
    g = o.grids[c]
    un = prim_to_cons(f(g.dof_x), 1.4)
    dt = 0.004
    exact = np.stack([prim_to_cons(f(g.dof_x, o.tb.tau[a] * dt), 1.4) for a in range(N + 1)])
    # the exact translation is a fixed point of eq:ader4 to round-off ...
    assert np.abs(o.predictor_map(c, exact, un, dt, 0.0) - exact).max() < 1e-13 * np.abs(exact).max()
    # ... and the iteration finds it to its tolerance
    q, it, ok = o.predictor(c, un, dt, 0.0)
    assert ok
    assert np.abs(q - exact).max() < 1e-11


def test_predictor_quadratic_field_exact_at_n2(mesh_3):
    """rho quadratic in x - u t: exact in the P2 space-time space."""
    o = Oracle(mesh_3, 2, Params(depth=8, tol=1e-12))
    vel = np.ones(3)

    def f(x, t=0.0):
        y = x - vel * t
        w = np.zeros((len(x), 5))
        w[:, 0] = 1.0 + 0.1 * y[:, 0] ** 2 - 0.05 * y[:, 1] * y[:, 2] + 0.2 * y[:, 2]
        w[:, 1:4] = vel
        w[:, 4] = 1.0
        return w
    c = 3
    g = o.grids[c]
    un = prim_to_cons(f(g.dof_x), 1.4)
    exact = np.stack([prim_to_cons(f(g.dof_x, o.tb.tau[a] * 0.004), 1.4) for a in range(3)])
    assert np.abs(o.predictor_map(c, exact, un, 0.004, 0.0) - exact).max() < 1e-13 * np.abs(exact).max()
    q, it, ok = o.predictor(c, un, 0.004, 0.0)
    assert ok
    assert np.abs(q - exact).max() < 1e-11


def test_anderson_and_plain_iteration_reach_the_same_fixed_point(mesh_3):
    o = Oracle(mesh_3, 2)
    u = o.initial_state(density_wave)
    dt = o.cfl_dt(u, 0.0005)
    for c in (0, 11):
        un = o.cell_state(u, c)
        qa, _, ok1 = o.predictor(c, un, dt, 0.0, depth=8, tol=1e-12)
        qp, _, ok2 = o.predictor(c, un, dt, 0.0, depth=0, tol=1e-12, max_iter=2000)
        assert ok1 and ok2
        assert np.abs(qa - qp).max() < 1e-11


@pytest.mark.parametrize("N", [1, 2])
def test_free_stream_preserved(mesh_3, N):
    o = Oracle(mesh_3, N)
    u = o.initial_state(lambda x: uniform_state(x))
    dt = o.cfl_dt(u, 0.004)
    u1, rep = o.step(u, dt)
    assert rep.converged and rep.positive
    assert np.abs(u1 - u).max() < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("N", [1, 2])
def test_conservation_and_density_wave_invariants(mesh_3, N):
    """sum_i 1^T M_i u_i is conserved on a periodic mesh; on the density wave
    velocity and pressure stay constant (every flux is affine in rho there)."""
    o = Oracle(mesh_3, N)
    u = o.initial_state(density_wave)
    dt = o.cfl_dt(u, 0.004)

    def totals(v):
        return np.array([sum(o.mass(c).sum(0) @ o.cell_state(v, c)[:, k] for c in range(o.n_cells))
                         for k in range(5)])
    t0 = totals(u)
    u1, rep = o.step(u, dt)
    u2, rep2 = o.step(u1, dt)
    assert rep.converged and rep2.converged
    assert np.abs(totals(u2) - t0).max() < 1e-14 * np.abs(t0).max() * 10
    w = cons_to_prim(u2.T, 1.4)
    assert np.abs(w[:, 1:4] - 1.0).max() < 1e-11
    assert np.abs(w[:, 4] - 1.0).max() < 1e-11
    assert np.abs(u2 - u).max() > 1e-6  # the wave did move


def test_rusanov_flux_antisymmetric_bit_exact(mesh_3):
    o = Oracle(mesh_3, 2)
    u = o.initial_state(density_wave)
    dt = o.cfl_dt(u, 0.004)
    _, rep = o.step(u, dt, keep=True)
    mus = rep.mu
    for c in range(o.n_cells):
        g = o.grids[c]
        for k in range(0, len(g.conn), 7):
            G = o.rusanov(c, k, rep.ti, mus, dt)
            nb, kn = int(g.nbr[k]), int(g.nbr_tri[k])
            Gn = o.rusanov(nb, kn, rep.ti, mus, dt)
            assert np.array_equal(G, -Gn[g.nbr_perm[k]])


def test_cfl_closed_form_uniform_state(mesh_3):
    o = Oracle(mesh_3, 2)
    prim = (1.3, 0.4, -0.3, 0.2, 0.9)
    u = o.initial_state(lambda x: uniform_state(x, prim))
    lam = math.sqrt(0.4 ** 2 + 0.3 ** 2 + 0.2 ** 2) + math.sqrt(1.4 * 0.9 / 1.3)
    hmin = min(g.h for g in o.grids.values())
    assert abs(o.cfl_dt(u, 0.3) - 0.3 * hmin / (5 * lam)) < 1e-15
    o2 = Oracle(mesh_3, 2, Params(mu=0.01))
    lam2 = max(lam + 2 * (4 * 0.01 / (3 * 1.3)) * 5 / g.h for g in o2.grids.values())
    assert abs(o2.cfl_dt(u, 0.3) - 0.3 * hmin / (5 * lam2)) < 1e-15


def test_detector_flags_compression_jump_only(mesh_4):
    """beta = 0 for a smooth state.  With velocity +1 in x for seeds in
    0 < x < 1/2 and -1 elsewhere, the flow converges on the plane x = 1/2 and
    diverges on x = 0: beta = 1 in every cell with a neighbour across the
    converging plane, beta = 0 where only the diverging plane or no jump is
    seen (Sec. 4.5)."""
    o = Oracle(mesh_4, 1, Params(av=True))
    u = o.initial_state(density_wave)
    assert all(o.detector(u, c)[0] == 0.0 for c in range(o.n_cells))
    seeds = mesh_4["seeds"]
    side = np.where(seeds[:, 0] < 0.5, 1.0, -1.0)
    u = np.zeros((5, o.ndof))
    for c, g in o.grids.items():
        w = np.tile([1.0, side[c], 0.0, 0.0, 1.0], (g.ndof, 1))
        u[:, o.dof_ptr[c]:o.dof_ptr[c + 1]] = prim_to_cons(w, 1.4).T
    n_comp = 0
    for c, g in o.grids.items():
        beta, mu = o.detector(u, c)
        comp = exp = False
        for nb in set(int(x) for x in g.nbr):
            if side[nb] == side[c]:
                continue
            dx = seeds[nb, 0] - seeds[c, 0]
            dx -= np.round(dx)
            # moving towards each other: left cell (+1) with a neighbour on its right
            if (side[c] > 0) == (dx > 0):
                comp = True
            else:
                exp = True
        if comp and not exp:
            assert beta == 1.0 and mu > 0.0
            n_comp += 1
        if exp and not comp:
            assert beta == 0.0 and mu == 0.0
        if not comp and not exp:
            assert beta == 0.0
    assert n_comp > 0
