"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Bars: integer connectivity bit-exact; state after whole
steps within 1e-12 relative L-infinity per conserved variable."""
import numpy as np
import pytest

from afe_inputs.fields import density_wave, smoothed_sphere, taylor_green_3d, uniform_state
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def rel_linf(a, b):
    """Relative L-infinity distance of two states: max|a - b| / max|b| over all
    conserved variables and DOFs."""
    return float(np.abs(a - b).max() / np.abs(b).max())


# Predictor stop on both sides.  The predictor is a fixed point defined up to
# its stop test; a step amplifies that ambiguity (density wave, 4^3 seeds,
# N = 2: 1.25e-12 apart at a stop of 1e-13, 2.8e-13 at 3e-14, 7.5e-14 at
# 1e-14), so parity is checked with both sides stopping at 1e-14, well below
# the 1e-12 bar.
TOL = 1e-14
# The artificial-viscosity case keeps 1e-13: its bar is derived from the
# oracle's own spread at that stop (see oracle_spread).
TOL_AV = 1e-13


def _run_both(mesh, N, field, steps, cfl, params_o, params_g, dt=None):
    from oracle.scheme import Oracle
    afe = _lib()
    params_o.tol = params_g.tol = TOL
    params_o.max_iter = params_g.max_iter = 600
    o = Oracle(mesh, N, params_o)
    u0 = o.initial_state(field)
    cd = afe.CellData(mesh, N, params_g)
    assert np.array_equal(cd.dof_ptr, o.dof_ptr)
    if dt is None:
        dt = o.cfl_dt(u0, cfl)
    ug = torch.tensor(u0, device="cuda")
    uo = u0.copy()
    reps = []
    for _ in range(steps):
        uo, rep = o.step(uo, dt)
        assert rep.converged and rep.positive
        reps.append(cd.step(ug, dt))
    return uo, ug.cpu().numpy(), reps, cd, o, dt


@pytest.mark.parametrize("N", [1, 2, 3])
def test_connectivity_bit_exact(mesh_4, N):
    from oracle.subgrid import build_cells
    afe = _lib()
    cd = afe.CellData(mesh_4, N)
    sp, conn, nb, perm = cd.connectivity()
    gs = build_cells(mesh_4, N)
    assert np.array_equal(conn, np.concatenate([gs[c].conn for c in range(mesh_4["n_cells"])]))
    assert np.array_equal(nb, np.concatenate([sp[gs[c].nbr] + gs[c].nbr_tri for c in range(mesh_4["n_cells"])]))
    assert np.array_equal(perm, np.concatenate([gs[c].nbr_perm for c in range(mesh_4["n_cells"])]))
    x = cd.dof_coords().cpu().numpy()
    xo = np.concatenate([gs[c].dof_x for c in range(mesh_4["n_cells"])]).T
    assert np.abs(x - xo).max() < 1e-14


def test_prim_to_cons_and_cfl(mesh_4):
    from oracle.physics import prim_to_cons
    from oracle.scheme import Oracle, Params
    afe = _lib()
    o = Oracle(mesh_4, 2, Params(mu=2e-3))
    cd = afe.CellData(mesh_4, 2, afe.Params(mu=2e-3))
    x = cd.dof_coords().cpu().numpy()
    prim = density_wave(np.mod(x.T, 1.0)).T.copy()
    ug = cd.prim_to_cons(torch.tensor(prim, device="cuda"))
    assert np.abs(ug.cpu().numpy() - prim_to_cons(prim.T, 1.4).T).max() < 1e-15 * 5
    uo = o.initial_state(density_wave)
    dto = o.cfl_dt(uo, 0.3)
    dtg = cd.cfl_dt(torch.tensor(uo, device="cuda"), 0.3)
    assert abs(dtg - dto) <= 1e-13 * dto


@pytest.mark.parametrize("N", [1, 2, 3])
def test_step_parity_density_wave(mesh_4, N):
    from oracle.scheme import Params
    afe = _lib()
    steps = 2 if N < 3 else 1
    uo, ug, reps, cd, o, dt = _run_both(mesh_4, N, density_wave, steps, 0.004, Params(), afe.Params())
    print(f"N={N}: iterations max {[r.iters_max for r in reps]}", flush=True)
    assert rel_linf(ug, uo) < 1e-12


def test_step_parity_history_drop(mesh_4):
    """A GPU history of 56 difference pairs against the oracle's 63 (N = 3,
    density wave; the stiffest cell needs about 63 iterations).  Once a cell
    holds 56 pairs the 8 oldest are dropped and the scaled Cholesky factor of
    the remaining 48 is rebuilt row by row (eq:ader4's fixed point does not
    depend on the history kept), so the state still meets the parity bar."""
    from oracle.scheme import Params
    afe = _lib()
    uo, ug, reps, cd, o, dt = _run_both(mesh_4, 3, density_wave, 1, 0.004, Params(), afe.Params(accel_depth=56))
    print(f"iterations max {reps[0].iters_max}; rel Linf {rel_linf(ug, uo):.2e}", flush=True)
    assert reps[0].iters_max > 57  # at least one cell dropped pairs and rebuilt its factor
    assert rel_linf(ug, uo) < 1e-12


def oracle_spread(mesh, N, u0, dt, steps, uref, **kw):
    """How precisely the oracle itself defines the result: relative L-infinity
    spread of u^{n+steps} over equally valid predictor iterations (Anderson
    depth 48 instead of 63, and a 3x tighter stop).  Where viscosity acts on
    thin sub-tetrahedra the step amplifies the part of the predictor error that
    the stopping test leaves along the stiffest modes."""
    from oracle.scheme import Oracle, Params
    spread = 0.0
    for extra in (dict(depth=48, tol=TOL_AV), dict(tol=TOL_AV / 3)):
        o = Oracle(mesh, N, Params(max_iter=600, **{**kw, **extra}))
        u = u0
        for _ in range(steps):
            u, rep = o.step(u, dt)
            assert rep.converged
        spread = max(spread, rel_linf(u, uref))
    return spread


def test_step_parity_with_artificial_viscosity(mesh_4):
    """Cells whose seed lies in r < 0.3 around the centre move outward at speed
    0.2 into gas at rest: cell-wise constant data, so the velocity jumps on the
    sphere's cell faces are compressive and the flattener switches the
    artificial viscosity on (Sec. 4.5).  The second step exercises the viscous
    predictor and corrector with the cell viscosities."""
    from oracle.physics import prim_to_cons
    from oracle.scheme import Oracle, Params
    afe = _lib()
    o = Oracle(mesh_4, 2, Params(av=True, tol=TOL_AV))
    seeds = mesh_4["seeds"]
    u0 = np.zeros((5, o.ndof))
    for c in range(o.n_cells):
        d = seeds[c] - 0.5
        r = np.linalg.norm(d)
        w = np.array([1.0, 0.0, 0.0, 0.0, 1.0]) if r >= 0.3 else np.array([1.0, *(0.2 * d / r), 1.0])
        u0[:, o.dof_ptr[c]:o.dof_ptr[c + 1]] = prim_to_cons(np.tile(w, (o.grids[c].ndof, 1)), 1.4).T
    dt = o.cfl_dt(u0, 0.004)
    cd = afe.CellData(mesh_4, 2, afe.Params(av=True, tol=TOL_AV))
    ug = torch.tensor(u0, device="cuda")
    uo = u0
    for _ in range(2):
        uo, rep = o.step(uo, dt)
        assert rep.converged and rep.positive
        r = cd.step(ug, dt)
    it, mu = cd.diagnostics()
    assert (mu > 0).any() and r.n_troubled > 0
    assert np.allclose(mu, [rep.mu[c] for c in range(o.n_cells)], rtol=1e-12, atol=0)
    # With mu_i ~ 0.1 on thin sub-tetrahedra the result is defined by the
    # predictor's stopping test only to ~1e-10: the bar is twice the oracle's
    # own spread over valid iterations, and at least 1e-12.
    spread = oracle_spread(mesh_4, 2, u0, dt, 2, uo, av=True)
    bar = max(1e-12, 2.0 * spread)
    assert spread < 1e-8
    assert rel_linf(ug.cpu().numpy(), uo) < bar


def test_step_parity_navier_stokes_taylor_green():
    from oracle.scheme import Params
    afe = _lib()
    box = 2 * np.pi
    mesh = periodic_voronoi(jittered_lattice_seeds(4, 0.25, 3, box=box), box=box)
    mu = 1.0 / 1600.0  # Re = 1600 with unit velocity and length scales
    field = lambda x: taylor_green_3d(x, mach=0.3)
    uo, ug, reps, cd, o, dt = _run_both(mesh, 2, field, 2, 0.004, Params(mu=mu), afe.Params(mu=mu))
    assert rel_linf(ug, uo) < 1e-12
    # the viscous terms do act at this level
    ue, _, _, _, _, _ = _run_both(mesh, 2, field, 2, 0.004, Params(), afe.Params(), dt=dt)
    assert rel_linf(ue, uo) > 1e-9


def test_step_parity_heat_conduction(mesh_4):
    """Navier-Stokes with heat conduction (mu = 1e-4, kappa = 5e-4, c_v = 2.5:
    Pr = 0.7) on the density wave, whose temperature varies: the temperature
    gradient enters the nodal energy flux, the time step and the face penalty
    (viscous eigenvalue kappa / (c_v rho)), one step at N = 2.  As with the
    artificial viscosity, the stiff diffusion on thin sub-tetrahedra amplifies
    what the stop test leaves of the predictor error, so the bar is twice the
    oracle's own spread between two equally valid stops (1e-14 and 1e-14 / 3),
    and at least 1e-12.  Measured: GPU 8.1e-13 from the oracle, its own spread
    5.4e-13, the oracle's 4.2e-13; after a second step both grow to ~1e-11."""
    from oracle.scheme import Oracle, Params
    afe = _lib()
    kw = dict(mu=1e-4, kappa=5e-4, cv=2.5)
    uo, ug, reps, cd, o, dt = _run_both(mesh_4, 2, density_wave, 1, 0.004, Params(**kw), afe.Params(**kw))
    o3 = Oracle(mesh_4, 2, Params(tol=TOL / 3, max_iter=600, **kw))
    u3, rep3 = o3.step(o3.initial_state(density_wave), dt)
    assert rep3.converged
    spread = rel_linf(u3, uo)
    print(f"GPU {rel_linf(ug, uo):.2e} from the oracle; oracle spread {spread:.2e}", flush=True)
    assert spread < 1e-10
    assert rel_linf(ug, uo) < max(1e-12, 2.0 * spread)
    # the heat flux does act at this level
    un, _, _, _, _, _ = _run_both(mesh_4, 2, density_wave, 1, 0.004, Params(mu=1e-4), afe.Params(mu=1e-4), dt=dt)
    assert rel_linf(un, uo) > 1e-9


def test_free_stream_and_conservation_on_gpu(mesh_4):
    from oracle.scheme import Oracle
    afe = _lib()
    o = Oracle(mesh_4, 2)
    cd = afe.CellData(mesh_4, 2)
    u0 = o.initial_state(lambda x: uniform_state(x))
    ug = torch.tensor(u0, device="cuda")
    dt = cd.cfl_dt(ug, 0.01)
    cd.step(ug, dt)
    assert np.abs(ug.cpu().numpy() - u0).max() < 1e-12 * np.abs(u0).max()
    u1 = o.initial_state(density_wave)
    mrow = [o.mass(c).sum(0) for c in range(o.n_cells)]

    def totals(v):
        return np.array([sum(mrow[c] @ o.cell_state(v, c)[:, k] for c in range(o.n_cells)) for k in range(5)])
    ug = torch.tensor(u1, device="cuda")
    for _ in range(3):
        cd.step(ug, dt)
    t0, t1 = totals(u1), totals(ug.cpu().numpy())
    assert np.abs(t1 - t0).max() < 1e-13 * np.abs(t0).max()


def test_failure_statuses(mesh_4):
    from oracle.scheme import Oracle
    afe = _lib()
    o = Oracle(mesh_4, 1)
    u0 = o.initial_state(density_wave)
    cd = afe.CellData(mesh_4, 1, afe.Params(max_iter=1, tol=1e-30))
    ug = torch.tensor(u0, device="cuda")
    with pytest.raises(afe.AfeError) as e:
        cd.step(ug, 1e-3)
    assert e.value.name == "AFE_E_NO_CONVERGENCE"
    bad = u0.copy()
    bad[4, 7] = 0.01  # energy below kinetic energy: negative pressure
    cd = afe.CellData(mesh_4, 1)
    ug = torch.tensor(bad, device="cuda")
    with pytest.raises(afe.AfeError) as e:
        cd.step(ug, 1e-4)
    assert e.value.name == "AFE_E_POSITIVITY"


@pytest.mark.parametrize("N", [2, 3])
def test_mixed_precision_reaches_the_fp64_fixed_point(mesh_4, N):
    """AFE_MIXED iterates with an FP32 M_i^-1 as preconditioner of the FP64
    residual of eq:ADER-localCauchy, so the step converges to the same fixed
    point: the state matches the FP64 oracle to the same bar."""
    from oracle.scheme import Params
    afe = _lib()
    steps = 2 if N < 3 else 1
    uo, ug, reps, cd, o, dt = _run_both(mesh_4, N, density_wave, steps, 0.004, Params(),
                                        afe.Params(precision=afe.AFE_MIXED))
    assert rel_linf(ug, uo) < 1e-12
