"""Distance of two states [5, ndof] used by the parity tests."""
import numpy as np

QUANTITIES = ("mass", "momentum", "energy")
_ROWS = (slice(0, 1), slice(1, 4), slice(4, 5))


def rel_linf_vars(a, b):
    """Relative L-infinity distance per conserved quantity of the Navier-Stokes
    system (Sec. 2): mass rho, momentum rho v (one vector: its three
    components share the scale max |rho v_i|, so a component that happens to
    be small is not judged against its own round-off) and energy rho E;
    max |a - b| / max |b| over the quantity's rows and all DOFs."""
    a = np.asarray(a)
    b = np.asarray(b)
    return np.array([float(np.abs(a[r] - b[r]).max() / np.abs(b[r]).max()) for r in _ROWS])


def rel_linf(a, b):
    """The largest of the per-quantity relative L-infinity distances."""
    return float(rel_linf_vars(a, b).max())
