"""Grundmann-Moeller quadrature on the reference tetrahedron (used for error
norms and as a brute-force check of the quadrature-free matrices).

Grundmann & Moeller (SIAM J. Numer. Anal. 15, 1978): for the n-simplex and
odd degree d = 2s + 1,
    int_T f = sum_{i=0}^{s} (-1)^i 2^{-2s} (d + n - 2i)^d / (i! (d + n - i)!)
              sum_{|beta| = s - i} f(x_beta),  x_beta barycentric (2 beta_j + 1)/(d + n - 2i),
over the unit simplex T (volume 1/n!).
"""
from __future__ import annotations

from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np


def _compositions(total: int, parts: int):
    for c in product(range(total + 1), repeat=parts):
        if sum(c) == total:
            yield c


@lru_cache(maxsize=None)
def tet_rule(degree: int):
    """Points [n, 3] and weights [n] on T^ (weights sum to 1/6), exact to `degree`."""
    n = 3
    s = max(0, (degree - 1 + 1) // 2)
    d = 2 * s + 1
    pts, wts = [], []
    for i in range(s + 1):
        w = (-1) ** i * 2.0 ** (-2 * s) * (d + n - 2 * i) ** d / (factorial(i) * factorial(d + n - i))
        for beta in _compositions(s - i, n + 1):
            lam = [(2 * b + 1) / (d + n - 2 * i) for b in beta]
            pts.append(lam[1:])
            wts.append(w)
    return np.array(pts), np.array(wts)


@lru_cache(maxsize=None)
def tri_rule(degree: int):
    """Same construction on the reference triangle (weights sum to 1/2)."""
    n = 2
    s = max(0, (degree - 1 + 1) // 2)
    d = 2 * s + 1
    pts, wts = [], []
    for i in range(s + 1):
        w = (-1) ** i * 2.0 ** (-2 * s) * (d + n - 2 * i) ** d / (factorial(i) * factorial(d + n - i))
        for beta in _compositions(s - i, n + 1):
            lam = [(2 * b + 1) / (d + n - 2 * i) for b in beta]
            pts.append(lam[1:])
            wts.append(w)
    return np.array(pts), np.array(wts)
