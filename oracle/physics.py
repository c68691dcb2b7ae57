"""Compressible Navier-Stokes closure (Sec. 2).

Conserved Q = (rho, rho v, rho E).  Flux tensor columns F_x = (f, g, h):
    mass      rho v
    momentum  rho v (x) v + sigma
    energy    v . (rho E I + sigma) - kappa grad T
with the Stokes stress sigma = (p + 2/3 mu div v) I - mu (grad v + grad v^T)
and the ideal-gas law p = (gamma - 1)(rho E - rho |v|^2 / 2).
The temperature is T = p / (rho R) with R = (gamma - 1) c_v, so
grad T = (grad e - v . grad v) / c_v with e = rho E / rho.  The paper's tests
neglect heat conduction (kappa = 0, the default here).  With
Pr = mu gamma c_v / kappa the second viscous eigenvalue gamma mu / (Pr rho) is
kappa / (c_v rho); the viscous eigenvalue used is the larger of it and
4 mu / (3 rho).

Arrays carry the 5 conserved variables in the last axis.
"""
from __future__ import annotations

import numpy as np


def prim_to_cons(w: np.ndarray, gamma: float) -> np.ndarray:
    """(rho, u, v, w, p) -> (rho, rho u, rho v, rho w, rho E)."""
    q = np.empty_like(w)
    rho = w[..., 0]
    vel = w[..., 1:4]
    q[..., 0] = rho
    q[..., 1:4] = rho[..., None] * vel
    q[..., 4] = w[..., 4] / (gamma - 1.0) + 0.5 * rho * (vel * vel).sum(-1)
    return q


def cons_to_prim(q: np.ndarray, gamma: float) -> np.ndarray:
    rho = q[..., 0]
    vel = q[..., 1:4] / rho[..., None]
    p = (gamma - 1.0) * (q[..., 4] - 0.5 * rho * (vel * vel).sum(-1))
    w = np.empty_like(q)
    w[..., 0] = rho
    w[..., 1:4] = vel
    w[..., 4] = p
    return w


def pressure(q: np.ndarray, gamma: float) -> np.ndarray:
    rho = q[..., 0]
    m = q[..., 1:4]
    return (gamma - 1.0) * (q[..., 4] - 0.5 * (m * m).sum(-1) / rho)


def sound_speed(q: np.ndarray, gamma: float) -> np.ndarray:
    """c = sqrt(gamma R T) = sqrt(gamma p / rho)."""
    return np.sqrt(gamma * pressure(q, gamma) / q[..., 0])


def flux(q: np.ndarray, gamma: float, mu: float = 0.0, grad_q: np.ndarray | None = None, kappa: float = 0.0,
         cv: float = 2.5) -> np.ndarray:
    """Physical flux F[..., x, v] (x = direction, v = conserved variable).

    q [..., 5]; grad_q [..., 3, 5] with grad_q[..., x, v] = d q_v / d x_x
    (needed only when mu != 0 or kappa != 0).
    """
    rho = q[..., 0]
    m = q[..., 1:4]
    E = q[..., 4]
    v = m / rho[..., None]
    p = (gamma - 1.0) * (E - 0.5 * (m * v).sum(-1))
    sigma = np.zeros(q.shape[:-1] + (3, 3))
    for i in range(3):
        sigma[..., i, i] = p
    if mu != 0.0:
        # grad v: dv_j/dx_i = (d m_j/dx_i - v_j d rho/dx_i) / rho
        gv = (grad_q[..., :, 1:4] - v[..., None, :] * grad_q[..., :, 0:1]) / rho[..., None, None]
        div = gv[..., 0, 0] + gv[..., 1, 1] + gv[..., 2, 2]
        sigma = sigma + (2.0 / 3.0) * mu * div[..., None, None] * np.eye(3) - mu * (gv + np.swapaxes(gv, -1, -2))
    F = np.empty(q.shape[:-1] + (3, 5))
    F[..., :, 0] = m
    F[..., :, 1:4] = rho[..., None, None] * v[..., :, None] * v[..., None, :] + sigma
    F[..., :, 4] = v * E[..., None] + (sigma * v[..., :, None]).sum(-2)
    if kappa != 0.0:
        # grad T = (grad e - v . grad v) / c_v, e = E / rho
        e = E / rho
        ge = (grad_q[..., :, 4] - e[..., None] * grad_q[..., :, 0]) / rho[..., None]
        gv = (grad_q[..., :, 1:4] - v[..., None, :] * grad_q[..., :, 0:1]) / rho[..., None, None]
        gT = (ge - (gv * v[..., None, :]).sum(-1)) / cv
        F[..., :, 4] -= kappa * gT
    return F


def max_eig(q: np.ndarray, gamma: float) -> np.ndarray:
    """Largest convective eigenvalue magnitude |v| + c."""
    rho = q[..., 0]
    vel = q[..., 1:4] / rho[..., None]
    return np.sqrt((vel * vel).sum(-1)) + sound_speed(q, gamma)


def visc_eig(q: np.ndarray, mu, kappa: float = 0.0, cv: float = 2.5) -> np.ndarray:
    """Largest viscous eigenvalue: max(4 mu / (3 rho), kappa / (c_v rho))."""
    return np.maximum(4.0 * mu / (3.0 * q[..., 0]), kappa / (cv * q[..., 0]))
