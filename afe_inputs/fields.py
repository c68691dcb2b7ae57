"""Analytic initial fields in primitive variables (rho, u, v, w, p).

Each function maps points x [n, 3] to an array [n, 5].  These are input
recipes only; conversion to conserved variables belongs to each solver.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def density_wave(x: np.ndarray, amp: float = 0.2, vel=(1.0, 1.0, 1.0), p0: float = 1.0,
                 t: float = 0.0, box: float = 1.0) -> np.ndarray:
    """rho = 1 + amp sin(2 pi (x + y + z - (u+v+w) t) / box), constant velocity and
    pressure.  An exact solution of the Euler equations (pure translation)."""
    x = np.asarray(x, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    phase = 2.0 * math.pi * ((x - vel * t) @ np.ones(3)) / box
    out = np.empty((len(x), 5))
    out[:, 0] = 1.0 + amp * np.sin(phase)
    out[:, 1:4] = vel
    out[:, 4] = p0
    return out


def smoothed_sphere(x: np.ndarray, radius: float, alpha: float, inner=(1.0, 1.0), outer=(0.125, 0.1),
                    centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Spherical Riemann problem with an erf-smoothed interface.

    Inside (rho, p) = inner, outside = outer, velocity zero; each primitive
    P = (P_out + P_in)/2 + (P_out - P_in)/2 * erf((r - R)/alpha), which tends
    to P_in for r << R and P_out for r >> R.
    """
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x - np.asarray(centre), axis=1)
    s = erf((r - radius) / alpha)
    out = np.zeros((len(x), 5))
    for col, (pin, pout) in ((0, (inner[0], outer[0])), (4, (inner[1], outer[1]))):
        out[:, col] = 0.5 * (pout + pin) + 0.5 * (pout - pin) * s
    return out


def taylor_green_3d(x: np.ndarray, mach: float = 0.1, gamma: float = 1.4) -> np.ndarray:
    """Classical 3D Taylor-Green vortex on [0, 2 pi]^3 with unit density:
    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16."""
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    out = np.empty((len(x), 5))
    out[:, 0] = 1.0
    out[:, 1] = np.sin(X) * np.cos(Y) * np.cos(Z)
    out[:, 2] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    out[:, 3] = 0.0
    out[:, 4] = 1.0 / (gamma * mach * mach) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    return out


def uniform_state(x: np.ndarray, prim=(1.0, 0.3, -0.2, 0.1, 1.0)) -> np.ndarray:
    """A constant state (free-stream)."""
    return np.tile(np.asarray(prim, dtype=np.float64), (len(x), 1))


def isentropic_vortex(x: np.ndarray, t: float = 0.0, strength: float = 5.0, centre=(5.0, 5.0),
                      vel=(0.0, 0.0, 0.0), gamma: float = 1.4) -> np.ndarray:
    """Two-dimensional isentropic vortex (Sec. 5.1-5.2): with r the distance
    from the centre (x_c + u_0 t, y_c + v_0 t) in the (x, y) plane and the
    temperature perturbation dT = -(gamma - 1) eps^2 / (8 gamma pi^2)
    exp(1 - r^2),
        rho = (1 + dT)^(1 / (gamma - 1)),  p = (1 + dT)^(gamma / (gamma - 1)),
        (u, v) = vel + eps / (2 pi) exp((1 - r^2) / 2) (-(y - y_c), x - x_c),
    w = vel_z.  With vel = 0 it is steady; with a constant background
    velocity it translates with it.  Exact for the Euler equations."""
    x = np.asarray(x, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    dx = x[:, 0] - (centre[0] + vel[0] * t)
    dy = x[:, 1] - (centre[1] + vel[1] * t)
    r2 = dx * dx + dy * dy
    dT = -(gamma - 1.0) * strength ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    a = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    out = np.empty((len(x), 5))
    out[:, 0] = (1.0 + dT) ** (1.0 / (gamma - 1.0))
    out[:, 1] = vel[0] - a * dy
    out[:, 2] = vel[1] + a * dx
    out[:, 3] = vel[2]
    out[:, 4] = (1.0 + dT) ** (gamma / (gamma - 1.0))
    return out


def affine_density(x: np.ndarray, t: float = 0.0, grad=(0.05, -0.03, 0.02), rho0: float = 1.0,
                   vel=(0.4, 0.3, -0.2), p0: float = 1.0) -> np.ndarray:
    """rho = rho0 + grad . (x - vel t), constant velocity and pressure: a
    translating density affine in space and time, an exact solution of the
    Euler equations (every flux is affine in rho at constant v and p)."""
    x = np.asarray(x, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    out = np.empty((len(x), 5))
    out[:, 0] = rho0 + (x - vel * t) @ np.asarray(grad, dtype=np.float64)
    out[:, 1:4] = vel
    out[:, 4] = p0
    return out


def shear_heating(x: np.ndarray, t: float = 0.0, a: float = 0.3, x0: float = 0.5, p0: float = 1.0,
                  mu: float = 0.01, gamma: float = 1.4) -> np.ndarray:
    """rho = 1, v = (0, a (x - x0), 0), p = p0 + (gamma - 1) mu a^2 t: a linear
    shear flow whose viscous dissipation heats the gas uniformly, an exact
    solution of the compressible Navier-Stokes equations (the stress is
    constant, the temperature uniform in space)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((len(x), 5))
    out[:, 0] = 1.0
    out[:, 2] = a * (x[:, 0] - x0)
    out[:, 4] = p0 + (gamma - 1.0) * mu * a * a * t
    return out


def shear_heating_grad(x: np.ndarray, t: float = 0.0, a: float = 0.3, **_) -> np.ndarray:
    """Gradient of shear_heating's primitive variables, [n, 3, 5] with
    [.., d, k] = d prim_k / d x_d."""
    g = np.zeros((len(x), 3, 5))
    g[:, 0, 2] = a
    return g


def stokes_first(x: np.ndarray, t: float = 0.0, nu: float = 1e-3, vl: float = 0.1, vr: float = -0.1,
                 t0: float = 0.05, gamma: float = 1.4) -> np.ndarray:
    """First problem of Stokes (Sec. 5.3): rho = 1, p = 1/gamma, u = w = 0,
    v = (vl + vr)/2 + (vr - vl)/2 erf((x - 1/2) / (2 sqrt(nu (t + t0)))), the
    incompressible shear-layer solution."""
    from scipy.special import erf
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((len(x), 5))
    out[:, 0] = 1.0
    out[:, 2] = 0.5 * (vl + vr) + 0.5 * (vr - vl) * erf((x[:, 0] - 0.5) / (2.0 * math.sqrt(nu * (t + t0))))
    out[:, 4] = 1.0 / gamma
    return out


def stokes_first_grad(x: np.ndarray, t: float = 0.0, nu: float = 1e-3, vl: float = 0.1, vr: float = -0.1,
                      t0: float = 0.05, **_) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    s = 2.0 * math.sqrt(nu * (t + t0))
    g = np.zeros((len(x), 3, 5))
    g[:, 0, 2] = 0.5 * (vr - vl) * 2.0 / math.sqrt(math.pi) * np.exp(-((x[:, 0] - 0.5) / s) ** 2) / s
    return g


def taylor_green_2d(x: np.ndarray, t: float = 0.0, nu: float = 1e-2, p0: float = 100.0) -> np.ndarray:
    """Two-dimensional Taylor-Green vortex (Sec. 5.5): rho = 1,
    u = sin x cos y e^(-2 nu t), v = -cos x sin y e^(-2 nu t), w = 0,
    p = p0 / gamma + (cos 2x + cos 2y) e^(-4 nu t) / 4 with gamma = 1.4 (the
    incompressible solution; p0 = 100 puts the Mach number near 0.1)."""
    x = np.asarray(x, dtype=np.float64)
    f = math.exp(-2.0 * nu * t)
    out = np.zeros((len(x), 5))
    out[:, 0] = 1.0
    out[:, 1] = np.sin(x[:, 0]) * np.cos(x[:, 1]) * f
    out[:, 2] = -np.cos(x[:, 0]) * np.sin(x[:, 1]) * f
    out[:, 4] = p0 / 1.4 + 0.25 * (np.cos(2 * x[:, 0]) + np.cos(2 * x[:, 1])) * f * f
    return out


def taylor_green_2d_grad(x: np.ndarray, t: float = 0.0, nu: float = 1e-2, **_) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    f = math.exp(-2.0 * nu * t)
    g = np.zeros((len(x), 3, 5))
    g[:, 0, 1] = np.cos(x[:, 0]) * np.cos(x[:, 1]) * f
    g[:, 1, 1] = -np.sin(x[:, 0]) * np.sin(x[:, 1]) * f
    g[:, 0, 2] = np.sin(x[:, 0]) * np.sin(x[:, 1]) * f
    g[:, 1, 2] = -np.cos(x[:, 0]) * np.cos(x[:, 1]) * f
    g[:, 0, 4] = -0.5 * np.sin(2 * x[:, 0]) * f * f
    g[:, 1, 4] = -0.5 * np.sin(2 * x[:, 1]) * f * f
    return g
