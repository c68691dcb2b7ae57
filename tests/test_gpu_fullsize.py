"""Parity at the full size of the throughput workload: the density wave on the
periodic Voronoi mesh of 16^3 jittered seeds (4096 cells, 2.35 M DOFs), N = 3,
one batched step with the time step from the CFL number on the device, in the
launch shape the throughput benchmark times (autotuned, eager, M^-1 profiling
on).  The oracle cannot step 4096 cells in seconds, so it steps sampled cells:
the largest cell (889 DOFs: 14 row tiles with a ragged last one), the smallest
and a seeded random one, with their face neighbours, whose predictors feed the
targets' face terms.  Bars: 1e-12 relative L-infinity on the sampled cells in
both precisions (stop test 1e-14 on both sides, as in the small parity tests);
the device time step equal to the oracle's over all cells (stored by
tests/golden/make_cfl_dt.py) to 1e-13; the default launch shape bit-identical
to the tuned one at this size."""
import dataclasses
import os

import numpy as np
import pytest

from afe_inputs.fields import density_wave
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from _metrics import rel_linf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
WL = dict(n=16, jitter=0.25, seed=1, N=3, cfl=0.004)
TOL = 1e-14


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def _golden_dt() -> float:
    with open(os.path.join(HERE, "golden", "wave16_p3_cfl_dt.txt")) as f:
        return float([ln for ln in f if not ln.startswith("#")][0])


@pytest.fixture(scope="module")
def oracle_step():
    """Mesh, sampled cells and the oracle's step of them from its own initial state."""
    from oracle.scheme import Oracle, Params, dof_counts
    _lib()
    mesh = periodic_voronoi(jittered_lattice_seeds(WL["n"], WL["jitter"], WL["seed"]))
    cnt = dof_counts(mesh, WL["N"])
    rnd = int(np.random.default_rng(7).integers(mesh["n_cells"]))
    targets = sorted({int(np.argmax(cnt)), int(np.argmin(cnt)), rnd})
    o = Oracle(mesh, WL["N"], Params(tol=TOL, max_iter=600), cells=targets)
    u0 = o.initial_state(density_wave)
    dt = _golden_dt()
    u1, rep = o.step(u0, dt)
    assert rep.converged and rep.positive
    print(f"targets {targets} (DOFs {[int(cnt[c]) for c in targets]}), ring {len(o.ring())} cells, "
          f"oracle iterations max {max(rep.iters.values())}", flush=True)
    return mesh, o, targets, u0, u1, dt


def _gpu_state(afe, cd, o, u0):
    """The device's own initial state, with the ring cells set to the oracle's."""
    x = cd.dof_coords().cpu().numpy()
    u = cd.prim_to_cons(torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda"))
    for c in o.ring():
        a, b = int(o.dof_ptr[c]), int(o.dof_ptr[c + 1])
        u[:, a:b] = torch.tensor(u0[:, a:b], device="cuda")
    return u


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_step_matches_oracle_on_sampled_cells(oracle_step, precision):
    afe = _lib()
    mesh, o, targets, u0, u1, dt = oracle_step
    p = afe.Params(tol=TOL, max_iter=600, precision=afe.AFE_MIXED if precision == "mixed" else afe.AFE_FP64)
    cd = afe.CellData(mesh, WL["N"], p)
    try:
        assert np.array_equal(cd.dof_ptr, o.dof_ptr)
        u = _gpu_state(afe, cd, o, u0)
        start = u.clone()
        b = afe.Batch()
        b.attach(cd, u, WL["cfl"])
        shape = b.tune()
        if shape.graph:
            shape = dataclasses.replace(shape, graph=False)
            b.shape = shape
        b.profile_enable(True)
        rep = b.step()[0]
        b.profile_enable(False)
        torch.cuda.synchronize()
        print(f"{precision}: shape {shape}, dt {rep.dt!r}, iterations {rep.iters_min}/{rep.iters_mean:.2f}/"
              f"{rep.iters_max}", flush=True)
        assert rep.status == "AFE_OK"
        assert abs(rep.dt - dt) <= 1e-13 * dt
        ug = u.cpu().numpy()
        for c in targets:
            a, e = int(o.dof_ptr[c]), int(o.dof_ptr[c + 1])
            err = rel_linf(ug[:, a:e], u1[:, a:e])
            print(f"  cell {c}: {e - a} DOFs, rel L-inf {err:.2e}", flush=True)
            assert err < 1e-12, c
        # the default launch shape gives the same bits at this size
        b.detach(cd)
        u2 = start.clone()
        b2 = afe.Batch()
        b2.attach(cd, u2, WL["cfl"])
        rep2 = b2.step()[0]
        torch.cuda.synchronize()
        assert rep2.dt == rep.dt and rep2.iters_max == rep.iters_max
        assert torch.equal(u2, u)
        b2.detach(cd)
    finally:
        cd.close()
        torch.cuda.empty_cache()
