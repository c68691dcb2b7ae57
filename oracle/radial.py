"""One-dimensional radial reference for the spherical explosion (Sec. 5.4).

Test infrastructure only, like the rest of `oracle/`.  Under spherical
symmetry the Euler equations of Sec. 2 (mu = 0) reduce to a problem in the
radius r; the paper obtains its reference solution with a second-order MUSCL
finite-volume scheme with the Rusanov flux on a radial mesh of 15,000 points
over [0, 1].  This module solves that problem plainly in float64:

    d/dt (r^a U) + d/dr (r^a F(U)) = (0, a r^(a-1) p, 0),
    U = (rho, rho u, E),  F = (rho u, rho u^2 + p, u (E + p)),

with a = 2 (sphere), or a = 0 (planar, the textbook shock tube used to pin
the scheme).  Cells [r_{i-1/2}, r_{i+1/2}] of equal width carry cell averages
with the volume weights V_i = (r_{i+1/2}^(a+1) - r_{i-1/2}^(a+1)) / (a+1) and
face areas A_{i+1/2} = r_{i+1/2}^a; the geometric pressure source is taken as
p_i (A_{i+1/2} - A_{i-1/2}), which balances the pressure flux of a gas at
rest exactly.  Reconstruction: primitive variables (rho, u, p), slopes limited
by minmod.  Time stepping: two-stage strong-stability-preserving Runge-Kutta
(Heun).  Boundaries: a reflecting wall at r = 0 (mirror cell with u -> -u) and
a transmissive one at r = r_max.
"""
from __future__ import annotations

import numpy as np


def _prim(U, gamma):
    rho = U[0]
    u = U[1] / rho
    p = (gamma - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


def _cons(rho, u, p, gamma):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _flux(rho, u, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.stack([rho * u, rho * u * u + p, u * (E + p)])


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


class RadialSolver:
    """Finite-volume solver on n equal cells over [0, r_max]."""

    def __init__(self, n: int, r_max: float = 1.0, geometry: int = 2, gamma: float = 1.4):
        self.n = n
        self.gamma = gamma
        self.a = geometry
        self.dr = r_max / n
        self.faces = np.arange(n + 1) * self.dr
        self.r = 0.5 * (self.faces[1:] + self.faces[:-1])
        a = geometry
        self.area = self.faces ** a
        self.vol = (self.faces[1:] ** (a + 1) - self.faces[:-1] ** (a + 1)) / (a + 1)

    def rhs(self, U):
        """Semi-discrete right-hand side dU/dt of the cell averages."""
        g = self.gamma
        rho, u, p = _prim(U, g)
        # ghost cells: mirror at r = 0, copy at r_max
        W = [np.concatenate([[q[0] * s], q, [q[-1]]]) for q, s in ((rho, 1.0), (u, -1.0), (p, 1.0))]
        left, right = [], []
        for q in W:
            d = _minmod(q[1:-1] - q[:-2], q[2:] - q[1:-1])  # slopes of the interior cells
            # the mirror cell's slope: rho and p are even in r (slope negated), u is odd (slope kept)
            d = np.concatenate([[d[0] if q is W[1] else -d[0]], d, [0.0]])
            # faces i + 1/2 for i = -1 .. n-1: left state from cell i, right from cell i+1
            left.append(q[:-1] + 0.5 * d[:-1])
            right.append(q[1:] - 0.5 * d[1:])
        rl, ul, pl = left
        rr, ur, pr = right
        Fl, Fr = _flux(rl, ul, pl, g), _flux(rr, ur, pr, g)
        Ul, Ur = _cons(rl, ul, pl, g), _cons(rr, ur, pr, g)
        s = np.maximum(np.abs(ul) + np.sqrt(g * pl / rl), np.abs(ur) + np.sqrt(g * pr / rr))
        F = 0.5 * (Fl + Fr) - 0.5 * s * (Ur - Ul)  # Rusanov flux at the n + 1 faces
        AF = F * self.area
        out = -(AF[:, 1:] - AF[:, :-1]) / self.vol
        out[1] += p * (self.area[1:] - self.area[:-1]) / self.vol
        return out

    def max_speed(self, U):
        rho, u, p = _prim(U, self.gamma)
        return float((np.abs(u) + np.sqrt(self.gamma * p / rho)).max())

    def run(self, rho0, u0, p0, t_end: float, cfl: float = 0.4):
        """Advance the initial primitive cell values to t_end; returns
        (rho, u, p) at the cell centres self.r."""
        U = _cons(np.asarray(rho0, float), np.asarray(u0, float), np.asarray(p0, float), self.gamma)
        t = 0.0
        while t < t_end:
            dt = min(cfl * self.dr / self.max_speed(U), t_end - t)
            U1 = U + dt * self.rhs(U)
            U = 0.5 * (U + U1 + dt * self.rhs(U1))
            t += dt
        return _prim(U, self.gamma)


def explosion_reference(t_end: float, radius: float, alpha: float, inner=(1.0, 1.0), outer=(0.125, 0.1),
                        n: int = 15000, r_max: float = 1.0, gamma: float = 1.4):
    """Radial solution of the spherical explosion with the erf-smoothed
    initial interface P = (P_in + P_out)/2 + (P_out - P_in)/2 erf((r - R)/alpha)
    for P = rho, p and zero velocity; returns (r, rho, u, p)."""
    from scipy.special import erf
    s = RadialSolver(n, r_max, 2, gamma)
    e = erf((s.r - radius) / alpha)
    rho0 = 0.5 * (outer[0] + inner[0]) + 0.5 * (outer[0] - inner[0]) * e
    p0 = 0.5 * (outer[1] + inner[1]) + 0.5 * (outer[1] - inner[1]) * e
    rho, u, p = s.run(rho0, np.zeros(n), p0, t_end)
    return s.r, rho, u, p


def signal_radius(t: float, radius: float, box: float = 1.0, speed: float = 2.5) -> float:
    """Largest radius around the centre that no wave from a periodic image of
    the sphere can have reached by time t: the nearest image interface lies at
    box - radius from the centre, and no signal travels faster than `speed`
    (above the shock speed of the standard states, about 1.75, and every
    |u| + c of the solution)."""
    return max(0.0, box - radius - speed * t)
