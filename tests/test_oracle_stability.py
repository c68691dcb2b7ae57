"""Stability probe of the step (power iteration of the linearised step) on the oracle.

On the density wave family (velocity (1,1,1), p = 1, rho = 1 + delta) every
flux is affine in rho and the uniform state is a fixed point of the step
(free stream), so the step maps delta linearly: delta^{n+1} = S delta^n.
Repeated steps of a seeded random delta (the power iteration of S,
renormalised each step) show whether a mode grows.  At the CFL number of the
workloads the perturbation stays bounded: after the transient growth of the
sub-grid noise it stops growing.  At a CFL number far above it the step is
not defined (the predictor does not reach its fixed point) or the
perturbation grows.  The same probe runs on the configured meshes through
the library (bench.py --stability)."""
import numpy as np

from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from oracle.physics import prim_to_cons
from oracle.scheme import Oracle, Params


def perturbation_growth(o, cfl, steps, eps=1e-2, seed=0):
    """Per-step growth factors of ||delta|| (None where the step fails)."""
    rng = np.random.default_rng(seed)
    delta = rng.uniform(-1.0, 1.0, o.ndof)
    base = np.zeros((o.ndof, 5))
    base[:, 0] = 1.0
    base[:, 1:4] = 1.0
    base[:, 4] = 1.0
    dt = o.cfl_dt(prim_to_cons(base, 1.4).T.copy(), cfl)
    out = []
    for _ in range(steps):
        w = base.copy()
        w[:, 0] = 1.0 + eps * delta / np.linalg.norm(delta)
        u1, rep = o.step(prim_to_cons(w, 1.4).T.copy(), dt)
        if not (rep.converged and rep.positive and np.isfinite(u1).all()):
            return out, False
        new = (u1[0] - 1.0) / eps
        out.append(float(np.linalg.norm(new)))
        delta = new
    return out, True


def test_perturbation_bounded_at_the_workload_cfl():
    mesh = periodic_voronoi(jittered_lattice_seeds(3, 0.2, 0))
    o = Oracle(mesh, 1, Params(tol=1e-12, max_iter=600))
    g, ok = perturbation_growth(o, 0.004, 80)
    assert ok
    amp = np.cumprod(g)
    tail = float(np.exp(np.mean(np.log(g[-20:]))))
    print(f"CFL 0.004: amplification {amp[-1]:.3f} after 80 steps (max {amp.max():.3f}), last 20 steps {tail:.5f}")
    assert amp.max() < 10.0 and tail < 1.01
    g2, ok2 = perturbation_growth(o, 1.0, 10)
    print(f"CFL 1.0: {'step fails' if not ok2 else 'growth %.3f' % np.exp(np.mean(np.log(g2)))}")
    assert (not ok2) or np.exp(np.mean(np.log(g2))) > 1.01
