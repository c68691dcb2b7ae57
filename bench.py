#!/usr/bin/env python3
"""Throughput of whole ADER-AFE-DG steps on one GPU (DOF-updates/s).

A step is one pass of the hot path: time step from the CFL condition with the
detector (Sec. 4.2, 4.5), space-time predictor (Sec. 4.3), quadrature-free
corrector with Rusanov faces and the positivity check (Sec. 4.4).  Inputs are
resident in device memory before the timed region.  Prints one JSON line.

Default workload: smooth density wave rho = 1 + 0.2 sin(2 pi (x+y+z)),
u = (1,1,1), p = 1 on the periodic Voronoi mesh of 16^3 jittered-lattice seeds
(+-0.25 h, seed 1), degree N = 3, FP64.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per ADER step, mixed vs FP64 at L2 err; p50/p99 solve latency"

WORKLOADS = {
    "wave16_p3": dict(n=16, jitter=0.25, seed=1, N=3, merge=None,
                      desc="density wave, periodic Voronoi 16^3 seeds (+-0.25h, seed 1), N=3, FP64"),
    "wave6_p2": dict(n=6, jitter=0.2, seed=0, N=2, merge=None,
                     desc="density wave, periodic Voronoi 6^3 seeds (+-0.2h, seed 0), N=2, FP64"),
    # the same seeds with Voronoi edges shorter than 2% of the seed spacing collapsed
    "wave16_p3_q": dict(n=16, jitter=0.25, seed=1, N=3, merge=0.02,
                        desc="density wave, periodic Voronoi 16^3 seeds (+-0.25h, seed 1), edges < 2% of "
                             "the seed spacing collapsed, N=3, FP64"),
}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the dominant kernels' own source text (the M^-1 tile routine and
    the FP64 and FP32 predictor launches): counters taken on them stay valid
    across unrelated edits, and become stale when these change."""
    with open(os.path.join(ROOT, "paper_2605_00619_amd", "csrc", "kernels.hip")) as fh:
        src = fh.read()
    h = hashlib.sha256()
    for sig in ("__device__ inline void minv_tile(", "k_round_minv(", "k_round_minv32("):
        i = src.index(sig)
        j = src.index("{", i)
        depth = 0
        for k in range(j, len(src)):
            depth += {"{": 1, "}": -1}.get(src[k], 0)
            if depth == 0:
                break
        h.update(src[i:k + 1].encode())
    return h.hexdigest()[:16]


def dominant_kernel(precision: str, N: int) -> str:
    nc = 5 * (N + 1)
    return f"k_round_minv<{nc}>" if precision == "fp64" else f"k_round_minv32<{nc}>"


def traffic_path(workload: str, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")


def measured_traffic(workload: str, precision: str, algorithmic_bytes_per_launch: float):
    """HBM bytes per launch of the dominant kernel: the ratio of counted to
    algorithmic bytes from committed counter runs, times this run's algorithmic
    bytes per launch; None unless the counters were taken on the current kernels."""
    path = traffic_path(workload, precision)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["hbm_over_algorithmic"] * algorithmic_bytes_per_launch


def summarize_counters(fetch_dir: str, write_dir: str) -> int:
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, each with --copy-probe-mib and its JSON line saved as
    bench.json in the output folder) into profiles/traffic_<workload>_<precision>.json.

    Each counter is calibrated on the plain 1 GiB device copy the run makes
    first (the largest __amd_rocclr_copyBuffer dispatch): factor = true bytes /
    counted bytes.  The dominant kernel's counted bytes, summed over its
    dispatches and scaled, are divided by the algorithmic bytes the library
    counted for the same dispatches."""
    import csv

    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        with open(os.path.join(d, "bench.json")) as fh:
            b = json.loads(fh.read().strip().splitlines()[-1])
        wl = b["config"]["name"]
        prec = "fp64" if b["dtype"] == "f64" else "mixed"
        name = dominant_kernel(prec, b["config"]["N"])
        copy_kib, kib, n = 0.0, 0.0, 0
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"):
                    copy_kib = max(copy_kib, v)
                elif name in r["Kernel_Name"]:
                    kib += v
                    n += 1
        true_kib = b["copy_probe_bytes"] / 1024.0
        factor = true_kib / copy_kib
        if n != b["roofline"]["launches"]:
            raise RuntimeError(f"{counter}: {n} dispatches of {name} counted, {b['roofline']['launches']} timed")
        alg = b["roofline"]["algorithmic_bytes_per_launch"] * n
        out[counter] = dict(counted_kib=kib, dispatches=n, copy_factor=factor,
                            bytes=kib * 1024.0 * factor, algorithmic_bytes=alg)
    rec = dict(workload=wl, precision=prec, kernel=name, kernel_source_hash=kernel_source_hash(),
               counters=out,
               hbm_over_algorithmic=sum(v["bytes"] for v in out.values()) / out["FETCH_SIZE"]["algorithmic_bytes"])
    with open(traffic_path(wl, prec), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))
    return 0


def host_description() -> dict:
    """Host cores as this process sees them and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def host_workers(cap: int = 16) -> int:
    """Worker processes for host-side preparation: the usable cores, at most cap."""
    return max(1, min(cap, len(os.sched_getaffinity(0))))


# state shared with forked oracle workers (set before each pool is created)
_CPU = {}


def _cpu_predict(c):
    """Predictor and time integrals of one cell (a forked worker, one thread)."""
    o, u0, dt = _CPU["o"], _CPU["u0"], _CPU["dt"]
    t0 = time.perf_counter()
    q, it, ok = o.predictor(c, o.cell_state(u0, c), dt, 0.0)
    ti = o.time_integrals(c, q, dt, 0.0)
    return c, ti, it, time.perf_counter() - t0


def _cpu_correct(c):
    """Corrector of one cell from the time integrals of it and its neighbours."""
    o, ti, dt = _CPU["o"], _CPU["ti"], _CPU["dt"]
    t0 = time.perf_counter()
    mus = {x: 0.0 for x in ti}
    rhs = ti[c]["vol"] - o.face_term(c, ti, mus, dt)
    o.mass_solve(c, rhs)
    return time.perf_counter() - t0


def cpu_baseline(mesh, N, u0_np, dt, gpu_iters_mean: float, cluster_size: int = 120, max_workers: int = 16):
    """Time the CPU oracle, unchanged, on a bounded sample of the same workload
    (same mesh, state and dt): predictor and time integrals on a cluster of
    cells (breadth-first from cell 0) and its face neighbours, then the
    corrector on the cluster.  Run twice on the same sample: one process with
    one thread, and one single-threaded process per usable host core (at most
    max_workers, the host share of one GPU), cells spread over the processes.
    DOF-updates/s = 5 x (sampled DOFs) / (wall time), per phase, so the figure
    is that of a whole step at the sample's per-DOF cost."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle.scheme import Oracle, Params

    n_cells = mesh["n_cells"]
    nbrs = [[] for _ in range(n_cells)]
    for a, b in mesh["face_cell"]:
        nbrs[int(a)].append(int(b))
        nbrs[int(b)].append(int(a))
    cluster, seen = [], {0}
    frontier = [0]
    while frontier and len(cluster) < cluster_size:
        c = frontier.pop(0)
        cluster.append(c)
        for x in nbrs[c]:
            if x not in seen:
                seen.add(x)
                frontier.append(x)
    o = Oracle(mesh, N, Params(), cells=cluster)
    ring = o.ring()
    dof_pred = sum(o.grids[c].ndof for c in ring)
    dof_corr = sum(o.grids[c].ndof for c in cluster)
    host = host_description()
    workers = max(1, min(max_workers, host["affinity"]))
    _CPU.update(o=o, u0=u0_np, dt=dt)
    out = {}
    with threadpool_limits(limits=1):
        for label, procs in (("1 core", 1), ("all cores", workers)):
            o._chol.clear()  # every run factorises its own mass matrices
            o._mass.clear()
            t0 = time.perf_counter()
            if procs == 1:
                res = [_cpu_predict(c) for c in ring]
            else:
                with mp.get_context("fork").Pool(procs) as pool:
                    res = pool.map(_cpu_predict, ring, chunksize=1)
            t_pred = time.perf_counter() - t0
            ti = {c: t for c, t, _, _ in res}
            iters = [it for _, _, it, _ in res]
            _CPU["ti"] = ti
            t0 = time.perf_counter()
            if procs == 1:
                for c in cluster:
                    _cpu_correct(c)
            else:
                with mp.get_context("fork").Pool(procs) as pool:
                    pool.map(_cpu_correct, cluster, chunksize=1)
            t_corr = time.perf_counter() - t0
            sec_per_dof = t_pred / dof_pred + t_corr / dof_corr
            out[label] = {"value": 5.0 / sec_per_dof, "processes": procs, "predictor_s": t_pred,
                          "corrector_s": t_corr, "oracle_iters_mean": float(sum(iters) / len(iters)),
                          "oracle_iters_max": int(max(iters))}
            log(f"cpu baseline [{label}]: {out[label]}")
    _CPU.clear()
    best = out["all cores"]
    return {
        "value": best["value"], "unit": "DOF-updates/s", "cores": best["processes"], "kind": "oracle",
        "one_core": out["1 core"], "all_cores": out["all cores"], "host": host,
        "gpu_iters_mean": gpu_iters_mean,
        "sample": (f"numpy FP64 oracle, one single-threaded process per core ({workers} of the "
                   f"{host['affinity']} usable host cores; also 1 core): predictor + time integrals on {len(ring)} "
                   f"cells ({dof_pred} DOFs), corrector on the {len(cluster)}-cell cluster they surround ({dof_corr} "
                   f"DOFs); same mesh, state and dt as the GPU run; the oracle starts every predictor from u^n "
                   f"(its mean iterations beside the GPU's); per-DOF cost taken as that of a whole step"),
    }


SERVE = dict(count=32, rate=20.0, seed=3, n_range=(4, 16), degrees=(2, 3), steps=20, cfl=0.004, mu=1.0 / 1600.0,
             merge=0.02, history_cells=256, reserve_gib=16,
             desc=("Navier-Stokes Taylor-Green vortex requests on [0, 2 pi)^3 (Mach 0.1, Re 1600, mixed precision), "
                   "periodic Voronoi of n^3 jittered seeds with edges < 2% of the spacing collapsed, n ~ U{4..16}, "
                   "N ~ U{2, 3}, 20 steps each, Poisson arrivals 20/s, 32 requests (seed 3), Anderson history pooled "
                   "(256 cells)"))


def serving_run(log) -> dict:
    """Continuous-batching session over the request stream; p50/p99 latency
    and aggregate DOF-updates/s."""
    import torch

    from afe_inputs.fields import taylor_green_3d
    from afe_inputs.requests import taylor_green_requests
    from paper_2605_00619_amd import afe
    from paper_2605_00619_amd.serve import GpuBackend, Request, Server, summarize

    t0 = time.time()
    raw = taylor_green_requests(SERVE["count"], SERVE["rate"], SERVE["seed"], SERVE["n_range"], SERVE["degrees"],
                                SERVE["steps"], merge=SERVE["merge"], workers=host_workers())
    log(f"serving: {len(raw)} request meshes in {time.time() - t0:.1f}s")
    params = afe.Params(mu=SERVE["mu"], precision=afe.AFE_MIXED, max_iter=400, history_cells=SERVE["history_cells"])
    reqs = [Request(d["rid"], d["arrival"], d["mesh"], d["N"], d["steps"], SERVE["cfl"], taylor_green_3d, params)
            for d in raw]
    free, _ = torch.cuda.mem_get_info()
    budget = free - SERVE["reserve_gib"] * 2**30
    srv = Server(GpuBackend(), budget)
    res = srv.run(reqs)
    out = summarize(res)
    out.update(workload=SERVE["desc"], hbm_budget_bytes=int(budget), peak_admitted_bytes=int(srv.peak_bytes),
               batch_steps=srv.steps_run, total_dofs=int(sum(r.ndof for r in res)),
               statuses=sorted({r.status for r in res}))
    log(f"serving: {out}")
    return out


BATCHED = dict(count=64, seed=2, cells=(500, 8000), degrees=(1, 2, 3), steps=50, cfl=0.004, merge=0.02,
               history_cells=256, reserve_gib=16,
               desc=("64 independent Euler runs (FP64) stepped as one batch: sizes ~ U{500..8000} cells realised as the "
                     "nearest cube n^3 of jittered seeds (+-0.25 h) with edges < 2% of the spacing collapsed, "
                     "N ~ U{1, 2, 3}, density wave or spherical Riemann problem (r < 0.3: rho = p = 1; else rho = "
                     "0.125, p = 0.1; erf-smoothed over 1.5 spacings, artificial viscosity on), 50 steps each at CFL "
                     "0.004, all arriving at t = 0, admitted by device memory (seed 2)"))


def batched_runs(log) -> dict:
    """The batched workload: 64 simulations of uneven sizes and degrees, all
    submitted at once to the continuous-batching server, which admits as
    many as device memory holds and steps them together (one launch per
    kernel over every admitted simulation's cells); DOF-updates/s over the
    whole session and the dominant kernel's bandwidth over its launches."""
    import numpy as np
    import torch

    from afe_inputs.fields import density_wave, smoothed_sphere
    from afe_inputs.requests import build_meshes
    from paper_2605_00619_amd import afe
    from paper_2605_00619_amd.serve import GpuBackend, Request, Server, summarize

    cfg = BATCHED
    rng = np.random.default_rng(cfg["seed"])
    sizes = rng.integers(cfg["cells"][0], cfg["cells"][1] + 1, size=cfg["count"])
    Ns = rng.choice(np.asarray(cfg["degrees"]), size=cfg["count"])
    sphere = rng.random(cfg["count"]) < 0.5
    mseeds = rng.integers(0, 2**31 - 1, size=cfg["count"])
    ns = [int(round(float(m) ** (1.0 / 3.0))) for m in sizes]
    t0 = time.time()
    meshes = build_meshes([(n, int(ms), 1.0, cfg["merge"]) for n, ms in zip(ns, mseeds)], host_workers())
    log(f"batched: {len(meshes)} meshes ({sum(m['n_cells'] for m in meshes)} cells) in {time.time() - t0:.1f}s")
    reqs = []
    for i, (mesh, N, sph, n) in enumerate(zip(meshes, Ns, sphere, ns)):
        if sph:
            field = (lambda a: (lambda x: smoothed_sphere(x, 0.3, a)))(1.5 / n)
        else:
            field = density_wave
        params = afe.Params(av=bool(sph), max_iter=400, history_cells=cfg["history_cells"])
        reqs.append(Request(i, 0.0, mesh, int(N), cfg["steps"], cfg["cfl"], field, params))
    free, _ = torch.cuda.mem_get_info()
    budget = free - cfg["reserve_gib"] * 2**30
    be = GpuBackend()
    be.batch.profile_enable(True)
    srv = Server(be, budget, setup_workers=4)
    res = srv.run(reqs)
    kms, launches, byts, stored = be.batch.profile_read()
    out = summarize(res)
    out.update(workload=cfg["desc"], hbm_budget_bytes=int(budget), peak_admitted_bytes=int(srv.peak_bytes),
               peak_active=srv.peak_active, batch_steps=srv.steps_run, total_dofs=int(sum(r.ndof for r in res)),
               statuses=sorted({r.status for r in res}),
               degrees={int(N): int((Ns == N).sum()) for N in cfg["degrees"]}, spheres=int(sphere.sum()),
               minv_kernel={"launches": int(launches), "ms": kms,
                            "achieved_GBps_packed": byts / (kms * 1e-3) / 1e9 if kms > 0 else None,
                            "achieved_GBps_as_stored": stored / (kms * 1e-3) / 1e9 if kms > 0 else None,
                            "note": "FP64 and FP32 M^-1 launches of all groups, algorithmic bytes on the packed basis"})
    log(f"batched: {out}")
    return out


def run_workload(args, key: str, precision: str, log, start=None, keep_initial: bool = False,
                 guess: bool = True) -> dict:
    """Build the workload, autotune the launch shape, run the warm-up and the
    timed steps with the M^-1 kernel's HIP events and byte counter."""
    import numpy as np
    import torch

    from afe_inputs.fields import density_wave
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    from paper_2605_00619_amd import afe

    wl = WORKLOADS[key]
    t0 = time.time()
    mesh = periodic_voronoi(jittered_lattice_seeds(wl["n"], wl["jitter"], wl["seed"]),
                            merge_tol=None if wl["merge"] is None else wl["merge"] / wl["n"])
    log(f"[{key} {precision}] mesh: {mesh['n_cells']} cells in {time.time() - t0:.1f}s")
    t0 = time.time()
    params = afe.Params(accel_depth=args.depth, max_iter=args.max_iter, tol=args.tol,
                        precision=afe.AFE_MIXED if precision == "mixed" else afe.AFE_FP64,
                        predictor_guess=guess and not args.no_guess)
    cd = afe.CellData(mesh, wl["N"], params)
    torch.cuda.synchronize()
    log(f"[{key} {precision}] cell data: ndof={cd.ndof} subtets={cd.n_subtets} max_cell_dofs={cd.max_cell_dofs} "
        f"device={cd.device_bytes / 2**30:.2f} GiB in {time.time() - t0:.1f}s")
    if start is None:
        x = cd.dof_coords()
        prim = torch.tensor(density_wave(np.mod(x.cpu().numpy().T, 1.0)).T.copy(), device="cuda")
        u = cd.prim_to_cons(prim)
        del x, prim
    else:
        u = start.clone()
    u_start = u.clone()
    batch = afe.Batch()
    batch.attach(cd, u, args.cfl)
    t0 = time.time()
    shape = batch.tune() if not args.no_tune else batch.shape
    log(f"[{key} {precision}] launch shape {shape} ({'tuned' if not args.no_tune else 'default'}) "
        f"in {time.time() - t0:.1f}s")
    if shape.graph:
        # the timed steps carry HIP events around the M^-1 launches, which graph replay would not
        shape = dataclasses.replace(shape, graph=False)
        batch.shape = shape
    for i in range(args.warmup):
        rep = batch.step()[0]
        log(f"[{key} {precision}] warmup {i}: dt={rep.dt:.3e} iters {rep.iters_min}/{rep.iters_mean:.1f}/{rep.iters_max}")
    torch.cuda.synchronize()
    batch.profile_enable(True)
    iters, iters_max = [], 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        rep = batch.step()[0]
        iters.append(rep.iters_mean)
        iters_max = max(iters_max, rep.iters_max)
        log(f"[{key} {precision}] step {i}: dt={rep.dt:.3e} iters {rep.iters_min}/{rep.iters_mean:.1f}/{rep.iters_max}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    k_ms, k_launches, k_bytes, k_stored = batch.profile_read()
    batch.profile_enable(False)
    achieved = (k_bytes / k_launches) / (k_ms / k_launches * 1e-3) / 1e9 if k_launches else None
    achieved_stored = (k_stored / k_launches) / (k_ms / k_launches * 1e-3) / 1e9 if k_launches else None
    res = {
        "value": cd.ndof * 5 * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
        "iters_mean": float(np.mean(iters)), "iters_max": int(iters_max), "dt": rep.dt,
        "cells": cd.n_cells, "ndof": cd.ndof, "subtets": cd.n_subtets, "mesh": mesh,
        "shape": {"sub": shape.sub, "minv": shape.minv, "anderson": shape.anderson, "rounds": shape.rounds,
                  "graph": bool(shape.graph)},
        "roofline": {
            "kernel": dominant_kernel(precision, wl["N"]) + (
                " (FP64 M_i^-1 applied to the predictor's space-time blocks)" if precision == "fp64" else
                " (FP32 scaled M_i^-1 applied to the predictor's residual blocks)"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(key, precision, k_bytes / max(k_launches, 1)),
            "avg_launch_ms": k_ms / max(k_launches, 1), "launches": k_launches,
            "algorithmic_bytes_per_launch": k_bytes / max(k_launches, 1),
            "algorithmic_bytes_basis": (
                "packed symmetric M_i^-1 (8 n_i (n_i+1)/2) + right-hand side read and result written "
                "(16 n_i 5(N+1)) per cell and iteration" if precision == "fp64" else
                "packed symmetric FP32 M_i^-1 (4 n_i (n_i+1)/2) + FP32 right-hand side read (4 n_i 5(N+1)) "
                "+ FP64 result written (8 n_i 5(N+1)) per cell and iteration"),
            "as_stored": {"achieved": achieved_stored, "frac": (achieved_stored / HBM_PEAK_GBS)
                          if achieved_stored else None, "bytes_per_launch": k_stored / max(k_launches, 1)},
            "share_of_step_time": (k_ms / 1e3) / elapsed,
            # the dominant kernel's algorithmic bytes over the whole step's time
            "step_frac": (k_bytes / elapsed / 1e9) / HBM_PEAK_GBS,
        },
        "u_end": u.clone(), "u_start": u_start if start is None else None,
        "u_initial": u_start if keep_initial else None,
    }
    batch.close()
    cd.close()
    del u
    torch.cuda.empty_cache()
    return res


def large_mesh_leg(log, steps: int = 5, history_cells: int = 2048) -> dict:
    """The spherical explosion (rho, p = 1, 1 inside r = 0.4, 0.125, 0.1 outside,
    erf width 0.01) with artificial viscosity on the 32^3-seed mesh (32768
    cells, +-0.25h, seed 1) with the Voronoi edges shorter than 2% of the seed
    spacing collapsed (complete linkage; on the diagram as it comes the
    stiffest cells' iteration count grows 136 -> 232 -> 249 over three steps),
    N = 3, in FP64 and in mixed precision from the same state, with the
    Anderson history pooled so that the object fits in HBM.  A few whole steps
    each: time per step, iterations, statuses, and the distance of the two
    final states."""
    import numpy as np
    import torch

    from afe_inputs.fields import smoothed_sphere
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    from paper_2605_00619_amd import afe

    t0 = time.time()
    from afe_inputs.requests import build_meshes
    mesh = build_meshes([(32, 1, 1.0, 0.02)])[0]  # complete linkage, a smaller tolerance if 2% does not close
    log(f"[explosion32_p3] mesh: {mesh['n_cells']} cells in {time.time() - t0:.1f}s")
    out, ends = {}, {}
    for prec in ("fp64", "mixed"):
        t0 = time.time()
        cd = afe.CellData(mesh, 3, afe.Params(av=True, max_iter=400, history_cells=history_cells,
                                               precision=afe.AFE_MIXED if prec == "mixed" else afe.AFE_FP64))
        torch.cuda.synchronize()
        setup = time.time() - t0
        x = cd.dof_coords().cpu().numpy()
        u = cd.prim_to_cons(torch.tensor(smoothed_sphere(np.mod(x.T, 1.0), 0.4, 0.01).T.copy(), device="cuda"))
        b = afe.Batch()
        b.attach(cd, u, 0.004)
        ms, reps = [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = b.step(check=False)[0]
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
            reps.append(r)
            log(f"[explosion32_p3 {prec}] {r.status} {ms[-1]:.1f} ms iters {r.iters_min}/{r.iters_mean:.2f}/"
                f"{r.iters_max} troubled {r.n_troubled}")
            if r.status != "AFE_OK":
                break
        out[prec] = {"ms_per_step": ms, "iters_mean": [r.iters_mean for r in reps],
                     "iters_max": [r.iters_max for r in reps], "status": [r.status for r in reps],
                     "n_troubled": [r.n_troubled for r in reps], "setup_s": setup,
                     "device_gib": cd.device_bytes / 2**30,
                     "dof_updates_per_s": cd.ndof * 5 / (np.mean(ms) * 1e-3)}
        out["ndof"] = cd.ndof
        ends[prec] = u.clone()
        b.close()
        cd.close()
        del u
        torch.cuda.empty_cache()
    if all(all(st == "AFE_OK" for st in out[p]["status"]) for p in ("fp64", "mixed")):
        out["mixed_rel_linf_vs_fp64"] = float((ends["mixed"] - ends["fp64"]).abs().max() / ends["fp64"].abs().max())
    out["workload"] = ("spherical explosion with artificial viscosity, periodic Voronoi 32^3 seeds (+-0.25h, seed 1), "
                       f"edges < 2% of the spacing collapsed, N=3, CFL 0.004, {steps} steps per precision, Anderson history pooled "
                       f"(history_cells={history_cells})")
    return out


STABILITY = {
    # configured meshes: (seeds per side, jitter, seed, N, steps per CFL number)
    "wave6_p2": (6, 0.2, 0, 2, 2000),
    "wave16_p3": (16, 0.25, 1, 3, 400),
}
STABILITY_CFL = (0.004, 0.008, 0.016, 0.03, 0.06, 0.12, 0.25, 0.5)


def stability_scan(log, keys=tuple(STABILITY), cfls=STABILITY_CFL, eps: float = 1e-3) -> dict:
    """CFL certification by the power iteration of the linearised step.  On
    the density wave family (velocity (1,1,1), p = 1, rho = 1 + delta) every
    flux is affine in rho and the uniform state is a fixed point of the step,
    so the step maps delta linearly.  From a seeded random delta, each step
    advances 1 + eps delta / ||delta|| and takes the new delta; the product of
    the norms' ratios is the amplification, the geometric mean over the last
    quarter of the steps the asymptotic growth per step.  A CFL number is
    certified when every step succeeds, the late growth is at most 1 + 1e-4
    and the amplification stays below 100 (transients of the sub-grid noise
    aside, no mode grows)."""
    import numpy as np
    import torch

    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    from paper_2605_00619_amd import afe

    out = {}
    for key in keys:
        n, jit, seed, N, steps = STABILITY[key]
        mesh = periodic_voronoi(jittered_lattice_seeds(n, jit, seed))
        cd = afe.CellData(mesh, N, afe.Params(max_iter=400))
        gen = torch.Generator(device="cuda").manual_seed(seed)
        base = torch.ones(5, cd.ndof, dtype=torch.float64, device="cuda")
        base[4] = 1.0 / 0.4 + 1.5
        rows = []
        for cfl in cfls:
            dt = cd.cfl_dt(base, cfl)
            d = torch.rand(cd.ndof, dtype=torch.float64, device="cuda", generator=gen) * 2.0 - 1.0
            norms, status, iters = [], "AFE_OK", 0
            t0 = time.time()
            for _ in range(steps):
                rho = 1.0 + eps * d / torch.linalg.vector_norm(d)
                u = torch.stack([rho, rho, rho, rho, 1.0 / 0.4 + 1.5 * rho]).contiguous()
                try:
                    rep = cd.step(u, dt)
                except afe.AfeError as e:
                    status = e.name
                    break
                iters = max(iters, rep.iters_max)
                d = (u[0] - 1.0) / eps
                norms.append(float(torch.linalg.vector_norm(d)))
            g = np.array(norms)
            amp = float(np.exp(np.cumsum(np.log(g))).max()) if len(g) else float("nan")
            q = max(1, len(g) // 4)
            late = float(np.exp(np.mean(np.log(g[-q:])))) if len(g) else float("nan")
            ok = status == "AFE_OK" and late <= 1.0 + 1e-4 and amp < 100.0
            rows.append({"cfl": cfl, "dt": dt, "steps": len(g), "status": status, "amplification_max": amp,
                         "late_growth_per_step": late, "predictor_iters_max": iters, "stable": ok})
            log(f"[stability {key}] CFL {cfl}: {rows[-1]} ({time.time() - t0:.1f}s)")
        certified = max([r["cfl"] for r in rows if r["stable"] and all(x["stable"] for x in rows if x["cfl"] <= r["cfl"])],
                        default=None)
        out[key] = {"cells": cd.n_cells, "N": N, "ndof": cd.ndof, "scan": rows, "certified_cfl": certified}
        cd.close()
        torch.cuda.empty_cache()
    return out


def configured_runs(log, cfl: float = 0.004, long_steps: int = 1000) -> dict:
    """Workloads run to their configured ends (density wave, FP64):
    - the 6^3-seed mesh (+-0.2 h, seed 0), N = 2, to t = 0.1: the L2 density
      error of Sec. 5 against the exact translated wave (afe_l2_error);
    - the 16^3-seed mesh (+-0.25 h, seed 1), N = 3, for long_steps steps: the
      largest predictor iteration count of every step (does the stiffest
      cells' count keep growing?) and the time per step."""
    import numpy as np
    import torch

    from afe_inputs.fields import density_wave
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    from paper_2605_00619_amd import afe

    out = {}
    mesh = periodic_voronoi(jittered_lattice_seeds(6, 0.2, 0))
    cd = afe.CellData(mesh, 2, afe.Params(max_iter=400))
    x = cd.dof_coords().cpu().numpy()
    u = cd.prim_to_cons(torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda"))
    t_end, t, steps, imax = 0.1, 0.0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end:
        dt = min(cd.cfl_dt(u, cfl), t_end - t)
        rep = cd.step(u, dt)
        t += dt
        steps += 1
        imax.append(rep.iters_max)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xq = cd.l2_points().cpu().numpy()
    err = cd.l2_error(u, 0, torch.tensor(density_wave(np.mod(xq, 1.0), t=t_end)[:, 0], device="cuda"))
    out["wave6_p2_to_t0.1"] = {"cells": cd.n_cells, "ndof": cd.ndof, "steps": steps, "cfl": cfl, "wall_s": wall,
                               "dof_updates_per_s": 5 * cd.ndof * steps / wall, "l2_density_error": err,
                               "iters_max_first_last": [imax[0], imax[-1]], "iters_max_max": int(max(imax))}
    log(f"[configured] {out['wave6_p2_to_t0.1']}")
    cd.close()
    mesh = periodic_voronoi(jittered_lattice_seeds(16, 0.25, 1))
    cd = afe.CellData(mesh, 3, afe.Params(max_iter=400))
    x = cd.dof_coords().cpu().numpy()
    u = cd.prim_to_cons(torch.tensor(density_wave(np.mod(x.T, 1.0)).T.copy(), device="cuda"))
    b = afe.Batch()
    b.attach(cd, u, cfl)
    imax, imean, t = [], [], 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(long_steps):
        r = b.step()[0]
        t += r.dt
        imax.append(r.iters_max)
        imean.append(r.iters_mean)
        if (k + 1) % 100 == 0:
            log(f"[configured] wave16_p3 step {k + 1}: t {t:.5f}, iterations max of the last 100 steps "
                f"{max(imax[-100:])}, mean {np.mean(imean[-100:]):.3f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xq = cd.l2_points().cpu().numpy()
    err = cd.l2_error(u, 0, torch.tensor(density_wave(np.mod(xq, 1.0), t=t)[:, 0], device="cuda"))
    blocks = [int(max(imax[i:i + 100])) for i in range(0, long_steps, 100)]
    out["wave16_p3_long"] = {"steps": long_steps, "t_end": t, "ms_per_step": 1e3 * wall / long_steps,
                             "dof_updates_per_s": 5 * cd.ndof * long_steps / wall,
                             "iters_max_per_100_steps": blocks, "iters_mean": float(np.mean(imean)),
                             "l2_density_error": err}
    log(f"[configured] {out['wave16_p3_long']}")
    b.close()
    cd.close()
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="wave16_p3", choices=sorted(WORKLOADS))
    ap.add_argument("--cfl", type=float, default=0.004)
    ap.add_argument("--depth", type=int, default=63)
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving session")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving session")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape instead of the autotuner's")
    ap.add_argument("--no-guess", action="store_true",
                    help="start every predictor iteration from u^n (default: from the previous step's predictor)")
    ap.add_argument("--no-large", action="store_true", help="skip the 32^3-seed explosion leg")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="skip the mixed-precision and mesh-variant legs")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--configured-runs", action="store_true",
                    help="only the density wave 6^3 N=2 to t=0.1 and 1000 steps of 16^3 N=3 (one JSON line)")
    ap.add_argument("--stability", action="store_true",
                    help="only the CFL certification scan of the configured meshes (one JSON line)")
    ap.add_argument("--batched-runs", action="store_true",
                    help="only the 64-simulation batched workload through the server (one JSON line)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic record from two counter runs and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters)
    if args.configured_runs:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(configured_runs(log)), flush=True)
        return 0
    if args.stability:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(stability_scan(log)), flush=True)
        return 0
    if args.batched_runs:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(batched_runs(log)), flush=True)
        return 0
    if args.serve_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serving_run(log)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the method is cell-local, a multi-GPU run would shard cells; not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from afe_inputs.fields import density_wave
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    from paper_2605_00619_amd import afe

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    copy_bytes = 0
    if args.copy_probe_mib:
        n = args.copy_probe_mib * 2**20 // 8
        copy_bytes = n * 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 8} bytes read, {n * 8} bytes written")
        del src, dst

    main_run = run_workload(args, args.workload, args.precision, log, keep_initial=not args.no_cpu_baseline)
    r = main_run
    out = {
        "metric": METRIC, "value": r["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (predictor preconditioner f32)",
        "data": "synthetic",
        "config": {
            "workload": wl["desc"], "name": args.workload, "cells": r["cells"], "ndof": r["ndof"],
            "subtets": r["subtets"], "N": wl["N"], "cfl": args.cfl, "dt_last": r["dt"],
            "predictor_iters_mean": r["iters_mean"], "predictor_iters_max": r["iters_max"],
            "anderson_depth": args.depth, "tol": args.tol, "launch_shape": r["shape"],
            "predictor_start": "u^n" if args.no_guess else
                               "previous step's predictor extrapolated in time (u^n on the first step)",
        },
        "copy_probe_bytes": copy_bytes,
        "roofline": r["roofline"],
    }
    if args.legs and args.precision == "fp64":
        # the same workload in mixed precision from the same initial state and the
        # same number of steps: throughput and distance of the final states
        mixed = run_workload(args, args.workload, "mixed", log, start=main_run["u_start"])
        diff = float((mixed["u_end"] - main_run["u_end"]).abs().max() / main_run["u_end"].abs().max())
        out["mixed"] = {k: mixed[k] for k in ("value", "ms_per_step", "iters_mean", "iters_max")}
        out["mixed"]["roofline"] = mixed["roofline"]
        out["mixed"]["rel_linf_vs_fp64_final_state"] = diff
        del mixed
        q = run_workload(args, "wave16_p3_q" if args.workload == "wave16_p3" else args.workload, "fp64", log)
        out["mesh_variant"] = {k: q[k] for k in ("value", "ms_per_step", "iters_mean", "iters_max", "ndof")}
        out["mesh_variant"]["workload"] = WORKLOADS["wave16_p3_q"]["desc"] if args.workload == "wave16_p3" else ""
        del q
        if not args.no_guess:
            # the same workload with every predictor iteration started from u^n
            p = run_workload(args, args.workload, "fp64", log, start=main_run["u_start"], guess=False)
            out["start_from_un"] = {k: p[k] for k in ("value", "ms_per_step", "iters_mean", "iters_max")}
            out["start_from_un"]["rel_linf_vs_main_final_state"] = float(
                (p["u_end"] - main_run["u_end"]).abs().max() / main_run["u_end"].abs().max())
            del p
    if args.legs and args.precision == "fp64" and not args.no_large:
        out["large_mesh"] = large_mesh_leg(log)
    u0_np = main_run["u_initial"].cpu().numpy() if main_run.get("u_initial") is not None else None
    mesh, dt = main_run["mesh"], main_run["dt"]
    del main_run, r
    if not args.no_serve:
        out["serving"] = serving_run(log)
    if not args.no_cpu_baseline:
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(mesh, wl["N"], u0_np, dt, out["config"]["predictor_iters_mean"])
        log(f"cpu baseline in {time.time() - t0:.1f}s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
