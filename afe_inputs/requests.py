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
                          steps: int = 10, merge: float | None = None, workers: int = 1) -> list[dict]:
    """`count` requests: arrival times (cumulative exponential gaps of mean
    1/rate), seeds per side n ~ U{n_range}, N ~ U{degrees}, mesh seed drawn
    per request; merge = collapse Voronoi edges shorter than merge times the
    seed spacing with complete linkage (None: the default merge of
    periodic_voronoi); workers > 1
    builds the meshes in that many forked processes (the draws and the
    meshes do not depend on it).  Returns dicts with rid, arrival, n, N,
    steps, mesh."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    Ns = rng.choice(np.asarray(degrees), size=count)
    mesh_seeds = rng.integers(0, 2**31 - 1, size=count)
    box = 2.0 * math.pi
    jobs = [(int(ns[i]), int(mesh_seeds[i]), box, merge) for i in range(count)]
    meshes = build_meshes(jobs, workers)
    out = []
    t = 0.0
    for i in range(count):
        t += float(gaps[i])
        out.append(dict(rid=i, arrival=t, n=int(ns[i]), N=int(Ns[i]), steps=steps, mesh=meshes[i]))
    return out


def _lattice_mesh(job):
    """With a collapse tolerance: complete-linkage merging, retried at half
    the tolerance while the diagram does not close (down to the default)."""
    n, mseed, box, merge = job
    seeds = jittered_lattice_seeds(n, 0.25, mseed, box=box)
    while merge is not None and merge > 1e-3:
        try:
            return periodic_voronoi(seeds, box=box, merge_tol=merge / n, linkage="complete")
        except RuntimeError:
            merge /= 2.0
    return periodic_voronoi(seeds, box=box)


def build_meshes(jobs, workers: int = 1) -> list[dict]:
    """Periodic Voronoi meshes of (n, mesh seed, box, merge) jittered
    lattices (+-0.25 h), in order, in `workers` forked processes (merge as in
    taylor_green_requests)."""
    if workers <= 1 or len(jobs) <= 1:
        return [_lattice_mesh(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
        return pool.map(_lattice_mesh, jobs, chunksize=1)
