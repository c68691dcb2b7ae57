"""Accuracy of the GPU path on the smooth density wave (an exact translating
solution of the Euler equations), measured with the error norm of Sec. 5
(the L2 norm of rho_h - rho_e, cell integrals over the sub-tetrahedra, by
the library's afe_l2_error): convergence with the mesh at degrees 2 and 3 on
the meshes as configured (Voronoi vertices merged per R11 only) and on the
variant with edges shorter than 2% of the seed spacing collapsed; the
mixed-precision path against FP64."""
import numpy as np
import pytest

from afe_inputs.fields import density_wave
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T_END = 0.01


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def l2_density_error(cd, u, t):
    xq = cd.l2_points().cpu().numpy()
    ref = torch.tensor(density_wave(np.mod(xq, 1.0), t=t)[:, 0], device="cuda")
    return cd.l2_error(u, 0, ref)


def _run(afe, n, N, precision, collapsed, T=T_END, cfl=0.004):
    mesh = periodic_voronoi(jittered_lattice_seeds(n, 0.25, 1), merge_tol=(0.02 / n) if collapsed else None)
    cd = afe.CellData(mesh, N, afe.Params(max_iter=400, precision=precision))
    x = cd.dof_coords().cpu().numpy()
    u = cd.prim_to_cons(torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda"))
    steps = int(np.ceil(T / cd.cfl_dt(u, cfl)))
    dt = T / steps
    for _ in range(steps):
        cd.step(u, dt, report=False)
    return l2_density_error(cd, u, T), steps


# Observed L2 orders 8^3 -> 16^3 seeds at t = 0.01; the paper's own L2 orders
# on its meshes run up to about 0.3 below N + 1 (its Tables 2-3).
@pytest.mark.parametrize("N,collapsed,bar", [(2, True, 2.5), (3, True, 3.5), (2, False, 2.5), (3, False, 3.5),
                                             (4, True, 4.5)])
def test_convergence_with_mesh(N, collapsed, bar):
    """Order of the L2 density error when the seed spacing halves, against
    the design order N + 1 less 0.5."""
    afe = _lib()
    e8, s8 = _run(afe, 8, N, afe.AFE_FP64, collapsed)
    e16, s16 = _run(afe, 16, N, afe.AFE_FP64, collapsed)
    p = np.log2(e8 / e16)
    print(f"N={N} {'collapsed' if collapsed else 'configured'}: L2 {e8:.3e} -> {e16:.3e}, order {p:.2f} "
          f"(design {N + 1}); steps {s8}, {s16}", flush=True)
    assert p >= bar


def test_mixed_precision_error_within_twice_fp64():
    """The mixed path converges to the FP64 fixed point, so its L2 error
    against the exact solution matches FP64's (bar: at most twice)."""
    afe = _lib()
    r64, _ = _run(afe, 8, 3, afe.AFE_FP64, True)
    rmx, _ = _run(afe, 8, 3, afe.AFE_MIXED, True)
    print(f"L2 error FP64 {r64:.6e}, mixed {rmx:.6e}", flush=True)
    assert rmx <= 2.0 * r64 and abs(rmx - r64) <= 1e-6 * r64
