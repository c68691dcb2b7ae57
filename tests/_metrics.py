"""Distance of two states [5, ndof] used by the parity tests."""
import numpy as np


def rel_linf_vars(a, b):
    """Relative L-infinity distance per conserved variable: max|a_v - b_v| /
    max|b_v| for v = rho, rho u, rho v, rho w, rho E.  A variable whose largest
    magnitude is below 1e-3 of the state's largest is measured against that
    1e-3 floor (a momentum component that is zero up to the step's own
    round-off has no scale of its own)."""
    a = np.asarray(a)
    b = np.asarray(b)
    floor = 1e-3 * float(np.abs(b).max())
    return np.array([float(np.abs(a[v] - b[v]).max() / max(float(np.abs(b[v]).max()), floor))
                     for v in range(b.shape[0])])


def rel_linf(a, b):
    """The largest of the per-variable relative L-infinity distances."""
    return float(rel_linf_vars(a, b).max())
