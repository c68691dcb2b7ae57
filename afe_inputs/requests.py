"""Seeded request streams for the serving workload (input recipe only).

Each request is a Taylor-Green vortex simulation on the periodic box
[0, 2 pi)^3 meshed by the Voronoi diagram of n^3 jittered lattice seeds
(+-0.25 h), with n and the degree N drawn per request; arrivals form a
Poisson process.  Everything is drawn from one numpy default_rng(seed).
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import jittered_lattice_seeds, periodic_voronoi


def taylor_green_requests(count: int, rate: float, seed: int, n_range=(4, 10), degrees=(2, 3),
                          steps: int = 10) -> list[dict]:
    """`count` requests: arrival times (cumulative exponential gaps of mean
    1/rate), seeds per side n ~ U{n_range}, N ~ U{degrees}, mesh seed drawn
    per request.  Returns dicts with rid, arrival, n, N, steps, mesh."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    Ns = rng.choice(np.asarray(degrees), size=count)
    mesh_seeds = rng.integers(0, 2**31 - 1, size=count)
    box = 2.0 * math.pi
    out = []
    t = 0.0
    for i in range(count):
        t += float(gaps[i])
        mesh = periodic_voronoi(jittered_lattice_seeds(int(ns[i]), 0.25, int(mesh_seeds[i]), box=box), box=box)
        out.append(dict(rid=i, arrival=t, n=int(ns[i]), N=int(Ns[i]), steps=steps, mesh=mesh))
    return out
