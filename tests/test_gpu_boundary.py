"""Bounded meshes with exact-solution Dirichlet data on the GPU (reading R21:
a boundary triangle's outside state is the exact solution at its face nodes
at the predictor's time nodes; Sec. 5.1-5.2 impose the exact solution on all
sides).

- The boundary face nodes the library lists are the oracle's face-node DOF
  coordinates of the boundary triangles, in ascending sub-tet order.
- An affine translating density is reproduced to round-off by one step
  (the closed form the oracle's pin also uses), N = 1, 2, 3.
- Parity with the oracle over two steps of the isentropic vortex travelling
  with the background flow (1, 1, 0), per conserved quantity, bar 1e-12.
- The allocation-free step equals the step bit for bit on a bounded mesh.
- Steady and travelling vortex (Sec. 5.1-5.2) on [0, 10]^2 x [0, 2.5]
  (collapsed short edges) with the Sec. 5 L2 density error: the error falls
  with the mesh at about the design order N + 1.
- Viscous data (the exact gradient with the state): a uniformly heated
  linear shear reproduced by one P3 step (with and without heat
  conduction); parity with the oracle on the first problem of Stokes (Sec.
  5.3); the 2D Taylor-Green vortex (Sec. 5.5) converging with the mesh.
- Misuse: a step without registered boundary states, a viscous step without
  their gradients and a batch attachment fail with AFE_E_ARG.
"""
import math

import numpy as np
import pytest

from afe_inputs.fields import (affine_density, isentropic_vortex, shear_heating, shear_heating_grad, stokes_first,
                               stokes_first_grad, taylor_green_2d, taylor_green_2d_grad)
from afe_inputs.mesh import box_voronoi, jittered_box_seeds
from _metrics import rel_linf_vars

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-14
SMALL_BOX = (1.0, 1.2, 0.9)


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def _fmt(v):
    return " ".join(f"{x:.1e}" for x in v)


def _small_mesh():
    return box_voronoi(jittered_box_seeds((3, 3, 3), SMALL_BOX, 0.25, 4), SMALL_BOX)


class Dirichlet:
    """Fills a CellData's boundary states with exact(x, t) (and, given grad,
    their gradients) at the boundary nodes and the predictor's time nodes of
    a step from t with step dt."""

    def __init__(self, cd, exact, grad=None):
        self.cd = cd
        self.exact = exact
        self.grad = grad
        self.x, self.tau = cd.boundary_nodes()
        self.buf = torch.empty((len(self.x), cd.N + 1, 5), dtype=torch.float64, device="cuda")
        cd.set_boundary_states(self.buf)
        if grad is not None:
            self.gbuf = torch.empty((len(self.x), cd.N + 1, 3, 5), dtype=torch.float64, device="cuda")
            cd.set_boundary_gradients(self.gbuf)

    def fill(self, t, dt):
        vals = np.stack([self.exact(self.x, t + ta * dt) for ta in self.tau], axis=1)
        self.buf.copy_(torch.from_numpy(np.ascontiguousarray(vals)))
        if self.grad is not None:
            gv = np.stack([self.grad(self.x, t + ta * dt) for ta in self.tau], axis=1)
            self.gbuf.copy_(torch.from_numpy(np.ascontiguousarray(gv)))


def test_boundary_nodes_are_the_oracle_face_nodes():
    from oracle.subgrid import build_cells
    afe = _lib()
    mesh = _small_mesh()
    for N in (1, 2, 3):
        cd = afe.CellData(mesh, N)
        x, tau = cd.boundary_nodes()
        gs = build_cells(mesh, N)
        xo = np.concatenate([gs[c].dof_x[gs[c].face_dof[k]] for c in range(mesh["n_cells"])
                             for k in range(len(gs[c].conn)) if gs[c].nbr[k] < 0])
        assert x.shape == xo.shape
        assert np.abs(x - xo).max() < 1e-14
        g = np.polynomial.legendre.leggauss(N + 1)[0]
        assert np.abs(tau - 0.5 * (g + 1.0)).max() < 1e-15


@pytest.mark.parametrize("N", [1, 2, 3])
def test_affine_solution_reproduced_on_gpu(N):
    afe = _lib()
    mesh = _small_mesh()
    exact = lambda x, t: affine_density(x, t, grad=(0.3, 0.2, 0.25), vel=(0.8, 0.5, 0.6))
    cd = afe.CellData(mesh, N, afe.Params(tol=TOL, max_iter=300))
    x = cd.dof_coords().cpu().numpy().T
    t0 = 0.3
    u = cd.prim_to_cons(torch.tensor(exact(x, t0).T.copy(), device="cuda"))
    u0 = u.clone()
    dt = 10.0 * cd.cfl_dt(u, 0.01)
    bc = Dirichlet(cd, exact)
    bc.fill(t0, dt)
    rep = cd.step(u, dt)
    ref = cd.prim_to_cons(torch.tensor(exact(x, t0 + dt).T.copy(), device="cuda"))
    err = float((u - ref).abs().max() / ref.abs().max())
    moved = float((u0 - ref).abs().max() / ref.abs().max())
    print(f"N={N}: moved {moved:.2e}, error {err:.2e}, iterations max {rep.iters_max}", flush=True)
    assert moved > 1e-4 and err < 1e-13


def test_step_parity_travelling_vortex():
    """Two steps from t = 0.1 on the small bounded mesh, N = 2, against the
    oracle stepped with the same boundary function."""
    from oracle.scheme import Oracle, Params as OParams
    afe = _lib()
    mesh = _small_mesh()
    N = 2
    exact = lambda x, t: isentropic_vortex(x, t, centre=(0.45, 0.55), vel=(1.0, 1.0, 0.0), strength=0.5)
    o = Oracle(mesh, N, OParams(tol=TOL, max_iter=600), boundary=exact)
    t = 0.1
    u0 = o.initial_state(lambda x: exact(x, t))
    dt = o.cfl_dt(u0, 0.004)
    cd = afe.CellData(mesh, N, afe.Params(tol=TOL, max_iter=600))
    ug = torch.tensor(u0, device="cuda")
    bc = Dirichlet(cd, exact)
    uo = u0.copy()
    for s in range(2):
        uo, rep = o.step(uo, dt, t=t + s * dt)
        assert rep.converged and rep.positive
        bc.fill(t + s * dt, dt)
        cd.step(ug, dt)
    err = rel_linf_vars(ug.cpu().numpy(), uo)
    print(f"travelling vortex, 2 steps: GPU vs oracle (mass, momentum, energy) {_fmt(err)}", flush=True)
    assert err.max() < 1e-12


def test_noalloc_step_equals_step_on_a_bounded_mesh():
    afe = _lib()
    mesh = _small_mesh()
    exact = lambda x, t: isentropic_vortex(x, t, centre=(0.45, 0.55), vel=(1.0, 1.0, 0.0), strength=0.5)
    outs = []
    for noalloc in (False, True):
        cd = afe.CellData(mesh, 2)
        x = cd.dof_coords().cpu().numpy().T
        u = cd.prim_to_cons(torch.tensor(exact(x, 0.0).T.copy(), device="cuda"))
        dt = cd.cfl_dt(u, 0.004)
        bc = Dirichlet(cd, exact)
        for s in range(2):
            bc.fill(s * dt, dt)
            (cd.step_noalloc if noalloc else cd.step)(u, dt)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy())
        cd.close()
    assert np.array_equal(outs[0], outs[1])


def test_bounded_mesh_misuse_fails():
    afe = _lib()
    mesh = _small_mesh()
    cdv = afe.CellData(mesh, 2, afe.Params(mu=0.01))
    x = cdv.dof_coords().cpu().numpy().T
    uv = cdv.prim_to_cons(torch.tensor(affine_density(x).T.copy(), device="cuda"))
    Dirichlet(cdv, lambda x, t: affine_density(x, t))  # states without gradients
    with pytest.raises(afe.AfeError) as e:
        cdv.step(uv, 1e-4)
    assert e.value.name == "AFE_E_ARG"
    cdv.close()
    cd = afe.CellData(mesh, 2)
    x = cd.dof_coords().cpu().numpy().T
    u = cd.prim_to_cons(torch.tensor(affine_density(x).T.copy(), device="cuda"))
    with pytest.raises(afe.AfeError) as e:
        cd.step(u, 1e-4)
    assert e.value.name == "AFE_E_ARG"
    b = afe.Batch()
    with pytest.raises(afe.AfeError) as e:
        b.attach(cd, u, 0.004)
    assert e.value.name == "AFE_E_ARG"
    b.close()
    with pytest.raises(ValueError):
        cd.set_boundary_states(torch.zeros((3, 3, 5), dtype=torch.float64, device="cuda"))


# ------------------------------------------------------------ vortex tests
VORTEX_BOX = (10.0, 10.0, 2.5)


def _vortex_run(afe, n, N, vel, t_end, cfl=0.004):
    """The isentropic vortex of strength 5 centred at (5, 5) (Sec. 5.1-5.2)
    on n x n x n/4 jittered seeds (+-0.25 h, seed 5) in [0, 10]^2 x [0, 2.5]
    with the edges shorter than 2% of the seed spacing collapsed (on the
    diagram as it comes, with edges down to 1e-3 of the spacing, a needle
    sub-tet next to the z = 0 plane carries a nodal error that grows until
    the 16 x 16 x 4 run fails its positivity check at t ~ 0.09, the sub-grid
    quality finding of the periodic meshes), exact Dirichlet data on all
    sides, to t_end; returns the Sec. 5 L2 density error and the number of
    steps."""
    exact = lambda x, t: isentropic_vortex(x, t, vel=vel)
    mesh = box_voronoi(jittered_box_seeds((n, n, max(1, n // 4)), VORTEX_BOX, 0.25, 5), VORTEX_BOX, merge_tol=0.02)
    cd = afe.CellData(mesh, N, afe.Params(max_iter=400))
    x = cd.dof_coords().cpu().numpy().T
    u = cd.prim_to_cons(torch.tensor(exact(x, 0.0).T.copy(), device="cuda"))
    bc = Dirichlet(cd, exact)
    steps = int(np.ceil(t_end / cd.cfl_dt(u, cfl)))
    dt = t_end / steps
    for s in range(steps):
        bc.fill(s * dt, dt)
        cd.step(u, dt, report=False)
    xq = cd.l2_points().cpu().numpy()
    ref = torch.tensor(exact(xq, t_end)[:, 0], device="cuda")
    err = cd.l2_error(u, 0, ref)
    cd.close()
    return err, steps


@pytest.mark.parametrize("N,vel", [(2, (0.0, 0.0, 0.0)), (2, (1.0, 1.0, 0.0)), (3, (1.0, 1.0, 0.0))])
def test_vortex_convergence(N, vel):
    afe = _lib()
    t_end = 0.2
    e1, s1 = _vortex_run(afe, 8, N, vel, t_end)
    e2, s2 = _vortex_run(afe, 16, N, vel, t_end)
    p = np.log2(e1 / e2)
    kind = "steady" if vel[0] == 0.0 else "travelling"
    print(f"{kind} vortex N={N} to t={t_end}: L2 {e1:.3e} -> {e2:.3e}, order {p:.2f} (design {N + 1}); "
          f"steps {s1}, {s2}", flush=True)
    # measured 2.73 (steady, N = 2), 2.69 (travelling, N = 2), 3.60 (N = 3);
    # the paper's L2 orders on its meshes are 2.73 / 3.99 (steady) and
    # 2.72 / 3.89 (travelling)
    assert p > N + 0.5


# ------------------------------------------------------ viscous boundary data
def _collapsed_small():
    return box_voronoi(jittered_box_seeds((3, 3, 3), SMALL_BOX, 0.25, 4), SMALL_BOX, merge_tol=0.02)


@pytest.mark.parametrize("kappa", [0.0, 0.02])
def test_viscous_shear_reproduced_on_gpu(kappa):
    """The oracle's viscous pin on the GPU: one P3 step of the uniformly heated
    linear shear with exact state and gradient as boundary data, against the
    exact solution (1e-11, the viscous stop's residue) and against the oracle
    per quantity within max(1e-12, 3 x the oracle's spread between stops of
    1e-14 and 1e-14 / 3), the bar of the other stiff parity cases."""
    from oracle.scheme import Oracle, Params as OParams
    afe = _lib()
    mesh = _collapsed_small()
    mu = 0.05
    exact = lambda x, t: shear_heating(x, t, a=0.8, mu=mu)
    grad = lambda x, t: shear_heating_grad(x, t, a=0.8)
    o = Oracle(mesh, 3, OParams(mu=mu, kappa=kappa, tol=TOL, max_iter=600), boundary=exact, boundary_grad=grad)
    t0 = 0.2
    u0 = o.initial_state(lambda x: exact(x, t0))
    dt = o.cfl_dt(u0, 0.004)
    uo, rep = o.step(u0, dt, t=t0)
    assert rep.converged
    o3 = Oracle(mesh, 3, OParams(mu=mu, kappa=kappa, tol=TOL / 3, max_iter=600), boundary=exact, boundary_grad=grad)
    uo3, rep3 = o3.step(u0, dt, t=t0)
    assert rep3.converged
    bar = np.maximum(1e-12, 3 * rel_linf_vars(uo3, uo))
    cd = afe.CellData(mesh, 3, afe.Params(mu=mu, kappa=kappa, tol=TOL, max_iter=600))
    ug = torch.tensor(u0, device="cuda")
    bc = Dirichlet(cd, exact, grad)
    bc.fill(t0, dt)
    cd.step(ug, dt)
    un = ug.cpu().numpy()
    ref = np.asarray(o.initial_state(lambda x: exact(x, t0 + dt)))
    err = float(np.abs(un - ref).max() / np.abs(ref).max())
    par = rel_linf_vars(un, uo)
    print(f"kappa={kappa}: error {err:.2e}; GPU vs oracle (mass, momentum, energy) {_fmt(par)}; bar {_fmt(bar)}",
          flush=True)
    assert err < 1e-11 and (par <= bar).all()


def test_step_parity_stokes_first_problem():
    """First problem of Stokes (Sec. 5.3, nu = 1e-2) on [0, 1] x [0, 0.2]^2
    (6 x 2 x 2 jittered seeds, short edges collapsed), N = 2, two steps from
    t = 0: GPU against oracle, per conserved quantity, within max(1e-12, 3 x
    the oracle's spread between stops of 1e-14 and 1e-14 / 3) (the momentum,
    0.1 at most, carries the viscous stop's ambiguity)."""
    from oracle.scheme import Oracle, Params as OParams
    afe = _lib()
    L = (1.0, 0.2, 0.2)
    mesh = box_voronoi(jittered_box_seeds((6, 2, 2), L, 0.25, 3), L, merge_tol=0.02)
    nu = 1e-2
    exact = lambda x, t: stokes_first(x, t, nu=nu)
    grad = lambda x, t: stokes_first_grad(x, t, nu=nu)
    o = Oracle(mesh, 2, OParams(mu=nu, tol=TOL, max_iter=600), boundary=exact, boundary_grad=grad)
    u0 = o.initial_state(lambda x: exact(x, 0.0))
    dt = o.cfl_dt(u0, 0.004)
    cd = afe.CellData(mesh, 2, afe.Params(mu=nu, tol=TOL, max_iter=600))
    ug = torch.tensor(u0, device="cuda")
    bc = Dirichlet(cd, exact, grad)
    o3 = Oracle(mesh, 2, OParams(mu=nu, tol=TOL / 3, max_iter=600), boundary=exact, boundary_grad=grad)
    uo = u0.copy()
    uo3 = u0.copy()
    for s in range(2):
        uo, rep = o.step(uo, dt, t=s * dt)
        uo3, rep3 = o3.step(uo3, dt, t=s * dt)
        assert rep.converged and rep.positive and rep3.converged
        bc.fill(s * dt, dt)
        cd.step(ug, dt)
    err = rel_linf_vars(ug.cpu().numpy(), uo)
    bar = np.maximum(1e-12, 3 * rel_linf_vars(uo3, uo))
    print(f"Stokes, 2 steps: GPU vs oracle (mass, momentum, energy) {_fmt(err)}; bar {_fmt(bar)}", flush=True)
    assert (err <= bar).all()


TG_BOX = (2 * math.pi, 2 * math.pi, math.pi / 2)


def _tg2d_run(afe, n, N, nu, t_end, cfl=0.004):
    """2D Taylor-Green vortex (Sec. 5.5, p0 = 100) on n x n x n/4 jittered
    seeds in [0, 2 pi]^2 x [0, pi/2] (short edges collapsed), exact state
    and gradient as boundary data on all sides, to t_end: the Sec. 5 L2 error
    of the x-momentum against rho u of the exact solution."""
    exact = lambda x, t: taylor_green_2d(x, t, nu=nu)
    grad = lambda x, t: taylor_green_2d_grad(x, t, nu=nu)
    mesh = box_voronoi(jittered_box_seeds((n, n, max(1, n // 4)), TG_BOX, 0.25, 6), TG_BOX, merge_tol=0.02)
    cd = afe.CellData(mesh, N, afe.Params(mu=nu, max_iter=400))
    x = cd.dof_coords().cpu().numpy().T
    u = cd.prim_to_cons(torch.tensor(exact(x, 0.0).T.copy(), device="cuda"))
    bc = Dirichlet(cd, exact, grad)
    steps = int(np.ceil(t_end / cd.cfl_dt(u, cfl)))
    dt = t_end / steps
    for s in range(steps):
        bc.fill(s * dt, dt)
        cd.step(u, dt, report=False)
    xq = cd.l2_points().cpu().numpy()
    w = exact(xq, t_end)
    err = cd.l2_error(u, 1, torch.tensor(w[:, 0] * w[:, 1], device="cuda"))
    cd.close()
    return err, steps


def test_taylor_green_2d_convergence():
    """Error of rho u at t = 0.05 (nu = 1e-2, N = 2) from 6 x 6 x 1 to
    10 x 10 x 2 seeds, order against the seed spacing.  Not every mesh of the
    family runs: with the viscous boundary data of R21 an oscillation grows at
    a boundary cell and fails the positivity check on 8 x 8 x 2, 11 x 11 x 2
    and 12 x 12 x 3 seeds at N = 2 and on every mesh beyond 6 x 6 x 1 at
    N = 3; the oracle shows the same growth (12 x 12 x 3, N = 2: the cell's
    smallest density 0.9992 -> 0.91 over steps 21-30, non-finite at 31), so it
    is the scheme under that reading, not the kernels."""
    afe = _lib()
    N = 2
    e1, s1 = _tg2d_run(afe, 6, N, 1e-2, 0.05)
    e2, s2 = _tg2d_run(afe, 10, N, 1e-2, 0.05)
    p = math.log(e1 / e2) / math.log(10 / 6)
    print(f"2D Taylor-Green N={N} to t=0.05: L2(rho u) {e1:.3e} -> {e2:.3e}, order {p:.2f} (design {N + 1}); "
          f"steps {s1}, {s2}", flush=True)
    assert p > N + 0.5
