"""The library's error norm (Sec. 5: the L2 norm of u_h - u_e summed over the
cells, each integral taken over the sub-tetrahedra): a closed form and the
oracle's own norm (a Grundmann-Moeller rule of degree 2N+3, an independent
quadrature) on the same state."""
import numpy as np
import pytest

from afe_inputs.fields import density_wave
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def _poly(x, N):
    """A polynomial of degree N in the cell-frame coordinates."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    p = 0.3 + 0.5 * X - 0.2 * Y + 0.1 * Z
    if N >= 2:
        p = p + 0.4 * X * Y - 0.3 * Z * Z
    if N >= 3:
        p = p + 0.2 * X * X * Z - 0.1 * Y * Y * Y
    return p


@pytest.mark.parametrize("N", [1, 2, 3])
def test_l2_norm_closed_form(mesh_4, N):
    """u_h[1] is the nodal interpolant of a polynomial p of degree N, so it is
    p itself on every sub-tet; against u_e = p + c the norm is |c| times the
    square root of the volume (the periodic unit box: 1), exactly up to
    round-off (the rule integrates degree 2N + 3)."""
    afe = _lib()
    print(f"N={N}", flush=True)
    cd = afe.CellData(mesh_4, N)
    x = cd.dof_coords().cpu().numpy().T
    u = np.zeros((5, cd.ndof))
    u[0] = 1.0
    u[1] = _poly(x, N)
    u[4] = 2.5
    ug = torch.tensor(u, device="cuda")
    xq = cd.l2_points().cpu().numpy()
    assert len(xq) == cd.n_subtets * (N + 3) ** 3
    for c in (0.0, 0.25):
        ref = torch.tensor(_poly(xq, N) + c, device="cuda")
        err = cd.l2_error(ug, 1, ref)
        print(f"  c={c}: {err!r}", flush=True)
        assert abs(err - c) < 1e-12


def test_l2_norm_matches_the_oracle(mesh_4):
    """The density wave after one step, N = 2: the library's norm against the
    exact wave and the oracle's (a Grundmann-Moeller rule and a conical product
    rule, both exact to degree 2N + 3; the integrand is not a polynomial, so
    they agree to the rules' error, not to round-off)."""
    from oracle.scheme import Oracle, Params
    afe = _lib()
    o = Oracle(mesh_4, 2, Params(tol=1e-14))
    u0 = o.initial_state(density_wave)
    dt = o.cfl_dt(u0, 0.004)
    uo, _ = o.step(u0, dt)
    eo = o.l2_error(uo, lambda x: density_wave(x, t=dt)[:, 0])
    cd = afe.CellData(mesh_4, 2)
    xq = cd.l2_points().cpu().numpy()
    ref = torch.tensor(density_wave(np.mod(xq, 1.0), t=dt)[:, 0], device="cuda")
    eg = cd.l2_error(torch.tensor(uo, device="cuda"), 0, ref)
    print(f"oracle {eo:.10e}, library {eg:.10e}, relative difference {abs(eg - eo) / eo:.2e}", flush=True)
    assert abs(eg - eo) < 1e-3 * eo
