"""The allocation-free step (ader_step_noalloc) against ader_step through the
C ABI: the same mesh, degree, state and time step on two separate objects,
two steps each, first on a 4^3-seed mesh and then, in the same process, on a
smaller 3^3-seed mesh (the device scratch array then holds the smaller
problem's lists over the larger one's).  The results must meet the parity bar
(1e-12 per conserved quantity); with the same kernels and launch shape they
are expected to be bit-identical."""
import numpy as np
import pytest

from _metrics import rel_linf
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


def _initial(afe, cd):
    x = cd.dof_coords().cpu().numpy()
    prim = torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda")
    return cd.prim_to_cons(prim)


def test_noalloc_step_equals_ader_step_on_two_sizes():
    afe = _lib()
    for n, seed, N in ((4, 0, 2), (3, 1, 2)):  # the second problem is the smaller one
        print(f"no-alloc vs ader_step: {n}^3 seeds (seed {seed}), N = {N}", flush=True)
        mesh = periodic_voronoi(jittered_lattice_seeds(n, 0.2, seed))
        a = afe.CellData(mesh, N)
        b = afe.CellData(mesh, N)
        ua = _initial(afe, a)
        ub = ua.clone()
        dt = a.cfl_dt(ua, 0.004)
        for step in range(2):
            ra = a.step_noalloc(ua, dt)
            rb = b.step(ub, dt)
            torch.cuda.synchronize()
            err = rel_linf(ua.cpu().numpy(), ub.cpu().numpy())
            same = bool(torch.equal(ua, ub))
            print(f"  step {step}: iterations {ra.iters_max}/{rb.iters_max}, rel L-inf {err:.1e}, "
                  f"bit-identical {same}", flush=True)
            assert (ra.iters_min, ra.iters_max, ra.n_troubled) == (rb.iters_min, rb.iters_max, rb.n_troubled)
            assert err < 1e-12
        a.close()
        b.close()


def test_noalloc_step_rejects_a_batched_object():
    afe = _lib()
    mesh = periodic_voronoi(jittered_lattice_seeds(3, 0.2, 0))
    cd = afe.CellData(mesh, 1)
    u = _initial(afe, cd)
    bt = afe.Batch()
    bt.attach(cd, u, 0.004)
    with pytest.raises(afe.AfeError) as e:
        cd.step_noalloc(u, 1e-4)
    assert e.value.name == "AFE_E_ARG"
    bt.close()
    cd.close()
