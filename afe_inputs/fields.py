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
