"""Accuracy of the GPU path on the smooth density wave (an exact translating
solution of the Euler equations): convergence with the mesh at degrees 2
and 3, and the mixed-precision path against FP64.

The meshes collapse Voronoi edges shorter than 2% of the seed spacing: on the
exact diagram, needle sub-tetrahedra under the shortest edges carry nodal
errors far above the bulk (the oracle shows the same), which hides the
order.  Errors are taken at the DOFs against the exact solution at the end
time; the density wave is interpolated exactly at the nodes at t = 0."""
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


def _run(afe, n, N, precision, T=T_END, cfl=0.004):
    mesh = periodic_voronoi(jittered_lattice_seeds(n, 0.25, 1), merge_tol=0.02 / n)
    cd = afe.CellData(mesh, N, afe.Params(max_iter=400, precision=precision))
    x = cd.dof_coords().cpu().numpy()
    u = cd.prim_to_cons(torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda"))
    steps = int(np.ceil(T / cd.cfl_dt(u, cfl)))
    dt = T / steps
    for _ in range(steps):
        cd.step(u, dt, report=False)
    e = u[0].cpu().numpy() - density_wave(np.mod(x.T, 1.0), t=T)[:, 0]
    return np.sqrt(np.mean(e * e)), np.median(np.abs(e)), steps


@pytest.mark.parametrize("N", [2, 3])
def test_convergence_with_mesh(N):
    """8^3 -> 16^3 seeds (h halves): RMS nodal error order >= N, median
    nodal error order >= N + 0.3 (measured 2.2 / 2.5 at N = 2, 3.5 / 3.7 at
    N = 3; the design order N+1 is approached from below on these irregular
    sub-grids)."""
    afe = _lib()
    r8, m8, s8 = _run(afe, 8, N, afe.AFE_FP64)
    r16, m16, s16 = _run(afe, 16, N, afe.AFE_FP64)
    p_rms, p_med = np.log2(r8 / r16), np.log2(m8 / m16)
    print(f"N={N}: rms {r8:.3e} -> {r16:.3e} (order {p_rms:.2f}), median {m8:.3e} -> {m16:.3e} "
          f"(order {p_med:.2f}); steps {s8}, {s16}", flush=True)
    assert p_rms >= N and p_med >= N + 0.3


def test_mixed_precision_error_within_twice_fp64():
    """The mixed path converges to the FP64 fixed point, so its error against
    the exact solution matches FP64's (bar: at most twice)."""
    afe = _lib()
    r64, m64, _ = _run(afe, 8, 3, afe.AFE_FP64)
    rmx, mmx, _ = _run(afe, 8, 3, afe.AFE_MIXED)
    print(f"rms error FP64 {r64:.6e}, mixed {rmx:.6e}", flush=True)
    assert rmx <= 2.0 * r64 and abs(rmx - r64) <= 1e-6 * r64
