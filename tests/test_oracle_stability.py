"""Stability probe of the step (the survey's test layer 6) on the oracle.

On the density wave family (velocity (1,1,1), p = 1, rho = 1 + delta) every
flux is affine in rho, the uniform state is a fixed point of the step
(free stream), so the step maps delta linearly: delta^{n+1} = S delta^n.  A
power iteration from a seeded random delta gives the growth factor of the
step's dominant mode; the step is stable at a CFL number where it is at
most 1.  Here on the 3^3-seed mesh at N = 1: stable at the CFL number the
workloads use, growing at a CFL number far above it."""
import numpy as np

from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from oracle.physics import prim_to_cons
from oracle.scheme import Oracle, Params


def step_growth(o, cfl, steps=40, tail=15, eps=1e-2, seed=0):
    """Geometric-mean growth of ||delta|| per step over the last `tail` steps."""
    rng = np.random.default_rng(seed)
    delta = rng.uniform(-1.0, 1.0, o.ndof)
    base = np.zeros((o.ndof, 5))
    base[:, 0] = 1.0
    base[:, 1:4] = 1.0
    base[:, 4] = 1.0
    dt = o.cfl_dt(prim_to_cons(base, 1.4).T.copy(), cfl)
    logs = []
    for _ in range(steps):
        w = base.copy()
        w[:, 0] = 1.0 + eps * delta / np.linalg.norm(delta)
        u1, rep = o.step(prim_to_cons(w, 1.4).T.copy(), dt)
        assert rep.converged and rep.positive
        new = (u1[0] - 1.0) / eps
        logs.append(np.log(np.linalg.norm(new)))
        delta = new
    return float(np.exp(np.mean(logs[-tail:])))


def test_step_stable_at_the_workload_cfl_and_growing_far_above():
    mesh = periodic_voronoi(jittered_lattice_seeds(3, 0.2, 0))
    o = Oracle(mesh, 1, Params(tol=1e-13, max_iter=600))
    g_small = step_growth(o, 0.004)
    g_large = step_growth(o, 1.0)
    print(f"growth per step: CFL 0.004 {g_small:.8f}, CFL 1.0 {g_large:.4f}")
    assert g_small <= 1.0 + 1e-9
    assert g_large > 1.0 + 1e-3
