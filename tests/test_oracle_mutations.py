"""The oracle's pins catch plausible mistakes.  Each case rebuilds one oracle
module from its source text with one deliberate change (in memory, on the
CPU), points the pin test at the changed module and expects the pin to fail:

- the sign of the (2/3) mu div v term of the Stokes stress (Sec. 2),
- the symmetric part of the velocity gradient replaced by 2 mu grad v,
- the viscous penalty 2 eps |lambda^v| dropped from the Rusanov flux (eq. 3.33),
- the face mass matrix Z^ lumped to its row sums (Sec. 4.4),
- the time weights w_a dropped from the predictor's stiffness term (eq:ader4),
- the boundary data taken at the start of the step instead of at the time
  nodes, or with the "+" side's own face nodes reversed, or the exact
  gradient left out of the viscous boundary flux (R21).
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import test_oracle_boundary as boundary_pins  # noqa: E402
import test_oracle_navier_stokes as pins  # noqa: E402
import test_oracle_scheme as scheme_pins  # noqa: E402


def _mutated(module: str, old: str, new: str):
    """A fresh copy of oracle.<module> whose source has `old` replaced by `new`."""
    path = os.path.join(os.path.dirname(oracle.__file__), module + ".py")
    with open(path) as fh:
        src = fh.read()
    assert src.count(old) == 1, (module, old)
    spec = importlib.util.spec_from_loader(f"oracle.{module}_mutated", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    sys.modules[spec.name] = mod  # dataclasses look their module up by name
    try:
        exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    finally:
        del sys.modules[spec.name]
    return mod


@pytest.fixture(scope="module")
def mesh3():
    return periodic_voronoi(jittered_lattice_seeds(3, 0.2, 0))


STRESS = [
    ("sign of the dilatation term", "sigma + (2.0 / 3.0) * mu", "sigma - (2.0 / 3.0) * mu",
     pins.test_stress_under_a_density_gradient_and_compression),
    ("2 mu grad v instead of mu (grad v + grad v^T)", "mu * (gv + np.swapaxes(gv, -1, -2))", "mu * (2.0 * gv)",
     pins.test_stress_simple_shear),
]


@pytest.mark.parametrize("name,old,new,pin", STRESS, ids=[s[0] for s in STRESS])
def test_stress_mutation_is_caught(monkeypatch, name, old, new, pin):
    pin()  # the pin holds on the oracle as it is
    mod = _mutated("physics", old, new)
    monkeypatch.setattr(pins, "flux", mod.flux)
    with pytest.raises(AssertionError):
        pin()


def test_dropped_viscous_penalty_is_caught(monkeypatch, mesh3):
    pins.test_rusanov_flux_two_states_at_rest(mesh3, 2)
    mod = _mutated("scheme", "s = lam + 2.0 * eps * lamv", "s = lam")
    monkeypatch.setattr(pins, "Oracle", mod.Oracle)
    with pytest.raises(AssertionError):
        pins.test_rusanov_flux_two_states_at_rest(mesh3, 2)


def test_lumped_face_mass_is_caught(monkeypatch):
    pins.test_face_mass_entrywise(2)
    mod = _mutated("refelem", "self.Z_f = f64(self.Z)", "self.Z_f = np.diag(f64(self.Z).sum(1))")
    monkeypatch.setattr(pins, "ref_element", mod.ref_element)
    with pytest.raises(AssertionError):
        pins.test_face_mass_entrywise(2)


def test_dropped_time_weights_are_caught(monkeypatch, mesh3):
    """Control: the predictor's closed-form pin sees the stiffness term's
    time weights."""
    scheme_pins.test_predictor_reproduces_translated_polynomial(mesh3, 2)
    mod = _mutated("scheme", 'np.einsum("a,k,dmp,akpdv->akmv", self.tb.w, g.detJ',
                   'np.einsum("a,k,dmp,akpdv->akmv", np.ones_like(self.tb.w), g.detJ')
    monkeypatch.setattr(scheme_pins, "Oracle", mod.Oracle)
    with pytest.raises(AssertionError):
        scheme_pins.test_predictor_reproduces_translated_polynomial(mesh3, 2)


BOUNDARY = [
    ("boundary data at t^n", "t = self.t + tau * dt", "t = self.t + 0.0 * tau * dt"),
    ("boundary face nodes reversed", "x = g.dof_x[g.face_dof[k]]", "x = g.dof_x[g.face_dof[k]][::-1]"),
]


@pytest.mark.parametrize("name,old,new", BOUNDARY, ids=[b[0] for b in BOUNDARY])
def test_boundary_mutation_is_caught(monkeypatch, name, old, new):
    boundary_pins.test_affine_solution_reproduced_with_boundary_data(2)
    mod = _mutated("scheme", old, new)
    monkeypatch.setattr(boundary_pins, "Oracle", mod.Oracle)
    with pytest.raises(AssertionError):
        boundary_pins.test_affine_solution_reproduced_with_boundary_data(2)


def test_dropped_boundary_gradient_is_caught(monkeypatch):
    """The viscous pin sees the gradient of the boundary data."""
    boundary_pins.test_viscous_shear_reproduced_with_boundary_data(0.0)
    mod = _mutated("scheme", "gw = self.boundary_grad(x, t)  # [nf, 3, 5]", "gw = 0.0 * self.boundary_grad(x, t)")
    monkeypatch.setattr(boundary_pins, "Oracle", mod.Oracle)
    with pytest.raises(AssertionError):
        boundary_pins.test_viscous_shear_reproduced_with_boundary_data(0.0)
