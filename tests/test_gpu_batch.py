"""Batched stepping through the C ABI (afe_batch_*): simulations of different
sizes, degrees and precisions share the predictor's launches.  Bars: a
simulation's state after batched steps is bit-identical to stepping it alone
(in a batch of one), for every launch shape; a batched step matches the CPU
oracle to 1e-12 relative L-infinity."""
import numpy as np
import pytest

from afe_inputs.fields import density_wave, smoothed_sphere
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
from _metrics import rel_linf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_00619_amd import afe
    afe.load()
    return afe


def _sphere(x):
    return smoothed_sphere(x, 0.3, 0.05)


# (seeds per side, jitter, seed, N, mixed, field, cfl, viscosity): uneven
# cell counts (27 to 125 cells), all three degrees, both precisions, two
# states; the last case is viscous, so that its degree group runs the viscous
# kernels for the inviscid case of the same degree too
CASES = [
    (3, 0.2, 0, 1, False, density_wave, 0.01, 0.0),
    (4, 0.2, 0, 2, False, density_wave, 0.004, 0.0),
    (5, 0.25, 3, 2, False, _sphere, 0.004, 0.0),
    (4, 0.25, 5, 3, True, density_wave, 0.004, 0.0),
    (4, 0.2, 7, 3, False, _sphere, 0.004, 0.0),
    (4, 0.2, 9, 2, False, density_wave, 0.004, 2e-3),
]


def _build(afe, case, tol=1e-12):
    n, jit, seed, N, mixed, field, cfl, mu = case
    mesh = periodic_voronoi(jittered_lattice_seeds(n, jit, seed))
    cd = afe.CellData(mesh, N, afe.Params(tol=tol, mu=mu, precision=afe.AFE_MIXED if mixed else afe.AFE_FP64))
    x = cd.dof_coords().cpu().numpy()
    prim = torch.tensor(field(np.mod(x.T, 1.0)).T.copy(), device="cuda")
    return mesh, cd, cd.prim_to_cons(prim), cfl


def _run(afe, cases, steps, shape=None):
    """Step `cases` together in one batch; returns their states and reports."""
    built = [_build(afe, c) for c in cases]
    b = afe.Batch()
    if shape is not None:
        b.shape = shape
    slots = [b.attach(cd, u, cfl) for (_, cd, u, cfl) in built]
    reps = [b.step() for _ in range(steps)]
    torch.cuda.synchronize()
    return [u.cpu().numpy() for (_, _, u, _) in built], [[r[s] for r in reps] for s in slots]


def test_batch_alone_equals_mixed():
    """Each simulation stepped in a batch with five others (packed cells of
    uneven counts, mixed degrees, precisions and viscosities) gives bit for
    bit the state it reaches alone, and the same time steps and iteration
    counts."""
    afe = _lib()
    mixed_u, mixed_r = _run(afe, CASES, steps=2)
    for i, case in enumerate(CASES):
        alone_u, alone_r = _run(afe, [case], steps=2)
        print(f"case {i}: N={case[3]} iters {[r.iters_mean for r in mixed_r[i]]}", flush=True)
        assert np.array_equal(alone_u[0], mixed_u[i]), f"case {i}"
        assert [r.dt for r in alone_r[0]] == [r.dt for r in mixed_r[i]]
        assert [r.iters_max for r in alone_r[0]] == [r.iters_max for r in mixed_r[i]]
        assert all(r.status == "AFE_OK" for r in mixed_r[i])


@pytest.mark.parametrize("shape", [
    dict(sub=0.0, minv=0.0, anderson=0.0, rounds=1, graph=False),
    dict(sub=2.0, minv=1.0, anderson=4.0, rounds=3, graph=False),
    dict(sub=1.0, minv=2.0, anderson=1.0, rounds=2, graph=True),
    dict(sub=1.0, minv=1.0, anderson=1.0, rounds=5, graph=True),
])
def test_batch_result_independent_of_launch_shape(shape):
    """Persistent or per-item grids, any number of iterations between reads,
    eager or graph replay (odd round counts exercise both list parities):
    the same bits."""
    afe = _lib()
    ref_u, ref_r = _run(afe, CASES[:4], steps=2)
    got_u, got_r = _run(afe, CASES[:4], steps=2, shape=afe.LaunchShape(**shape))
    for i in range(4):
        assert np.array_equal(ref_u[i], got_u[i]), f"case {i}"
        assert [r.iters_mean for r in ref_r[i]] == [r.iters_mean for r in got_r[i]]


def test_batch_tuner_keeps_states_and_results():
    afe = _lib()
    built = [_build(afe, c) for c in CASES[1:4]]
    b = afe.Batch()
    for (_, cd, u, cfl) in built:
        b.attach(cd, u, cfl)
    before = [u.clone() for (_, _, u, _) in built]
    chosen = b.tune()
    torch.cuda.synchronize()
    print("tuned shape", chosen, flush=True)
    for u0, (_, _, u, _) in zip(before, built):
        assert torch.equal(u0, u)
    assert b.shape == chosen
    b.step()
    ref_u, _ = _run(afe, CASES[1:4], steps=1)
    for i, (_, _, u, _) in enumerate(built):
        assert np.array_equal(u.cpu().numpy(), ref_u[i])


def test_batch_step_matches_oracle():
    """A batched step (time step from the CFL number on the device) against
    the oracle's step at the oracle's own CFL time step."""
    from oracle.scheme import Oracle, Params
    afe = _lib()
    tol = 1e-14  # both sides, far below the bar (the fixed point is defined up to the stop test)
    mesh = periodic_voronoi(jittered_lattice_seeds(4, 0.2, 0))
    o = Oracle(mesh, 2, Params(tol=tol, max_iter=600))
    u0 = o.initial_state(density_wave)
    dt = o.cfl_dt(u0, 0.004)
    uo, rep = o.step(u0, dt)
    assert rep.converged
    other = _build(afe, CASES[0])
    cd = afe.CellData(mesh, 2, afe.Params(tol=tol, max_iter=600))
    ug = torch.tensor(u0, device="cuda")
    b = afe.Batch()
    b.attach(other[1], other[2], other[3])
    s = b.attach(cd, ug, 0.004)
    r = b.step()[s]
    assert abs(r.dt - dt) <= 1e-13 * dt
    assert rel_linf(ug.cpu().numpy(), uo) < 1e-12


def test_batch_attach_errors_and_detach():
    afe = _lib()
    _, cd, u, cfl = _build(afe, CASES[0])
    b = afe.Batch()
    b.attach(cd, u, cfl)
    with pytest.raises(afe.AfeError) as e:
        b.attach(cd, u, cfl)
    assert e.value.name == "AFE_E_ARG"
    with pytest.raises(afe.AfeError):
        afe.Batch().attach(cd, u, cfl)
    b.detach(cd)
    assert b.step() == {}
    b2 = afe.Batch()
    b2.attach(cd, u, cfl)
    assert b2.step()[0].status == "AFE_OK"


def test_estimate_bytes_matches_allocation():
    """The host-side closed-form estimate used for admission equals what the
    object allocates, up to the allocator's per-buffer minimum."""
    afe = _lib()
    for case in CASES:
        n, jit, seed, N, mixed, _, _, mu = case
        mesh = periodic_voronoi(jittered_lattice_seeds(n, jit, seed))
        p = afe.Params(mu=mu, precision=afe.AFE_MIXED if mixed else afe.AFE_FP64)
        est = afe.estimate_bytes(mesh, N, p)
        cd = afe.CellData(mesh, N, p)
        assert abs(est - cd.device_bytes) <= 0.02 * cd.device_bytes, (case, est, cd.device_bytes)


def test_early_passes_do_not_change_bits():
    """On 512 cells the time-integral and corrector passes start while a few
    cells still iterate (at 1/16 and 1/256 of the cells); batched with another
    simulation the passes start at other iterations.  The states are bit
    identical, over three steps."""
    afe = _lib()
    big = (8, 0.25, 4, 2, False, density_wave, 0.004, 0.0)
    other = (6, 0.2, 5, 2, False, _sphere, 0.004, 0.0)
    alone_u, alone_r = _run(afe, [big], steps=3)
    mixed_u, mixed_r = _run(afe, [big, other], steps=3)
    print("iterations", [(r.iters_mean, r.iters_max) for r in alone_r[0]], flush=True)
    assert np.array_equal(alone_u[0], mixed_u[0])
    assert [r.iters_max for r in alone_r[0]] == [r.iters_max for r in mixed_r[0]]
