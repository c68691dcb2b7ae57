"""Serving loop: simulations as requests, continuously batched on one GPU.

A request is a whole simulation (mesh, degree, parameters, initial field,
CFL number, number of steps).  The loop admits requests in arrival order
while a batch slot is free and the device-memory estimate of the request
(afe_estimate_bytes plus its state) fits in what the budget has left;
admitted requests are set up (sub-grid, inverse mass matrices, initial
state) on worker threads, each with a stream of its own, overlapping the steps
of the running batch, then join the batch at the next step boundary.  Every
batch step advances all joined simulations by one ADER step; a simulation
leaves (slot and memory released) after its last step or when a step fails.
States stay resident on the device from setup to completion.

Latency of a request = completion - arrival, split into queue (waiting for
admission), setup and solve.  The scheduling logic talks to a backend
(estimate / setup / attach / step / release, and discard for a set-up
request that the batch refused) so that it can be exercised without a GPU;
GpuBackend is the libafe one.  A request whose set-up or join fails is
retired with the error's status and its memory returned to the budget; the
rest of the batch keeps running.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import threading
import time
from dataclasses import dataclass, field
from typing import Callable

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                      # seconds after the session start
    mesh: dict
    N: int
    steps: int
    cfl: float
    field: Callable[[np.ndarray], np.ndarray]  # primitive variables at points [n, 3] -> [n, 5]
    params: object = None               # afe.Params (None: defaults)


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    ready: float = float("nan")
    done: float = float("nan")
    ndof: int = 0
    steps_done: int = 0
    status: str = "AFE_OK"
    bytes: int = 0
    state: object = None                # final state (kept when requested)
    iters_mean: list = field(default_factory=list)

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queue(self) -> float:
        return self.admitted - self.arrival

    @property
    def setup(self) -> float:
        return self.ready - self.admitted

    @property
    def solve(self) -> float:
        return self.done - self.ready


class GpuBackend:
    """libafe on the current GPU: a Batch stepped on its own stream, set-ups
    on one stream per worker thread."""

    def __init__(self, shape=None):
        import torch

        from . import afe
        self.afe = afe
        self.torch = torch
        self.batch = afe.Batch()
        if shape is not None:
            self.batch.shape = shape
        self.local = threading.local()  # one set-up stream per worker thread
        self.step_stream = torch.cuda.Stream()

    def estimate(self, req: Request) -> int:
        """Library estimate plus the resident state and the set-up
        temporaries (DOF coordinates, primitive copy): 13 doubles per DOF,
        bounded by the DOFs of all sub-tet nodes (np per sub-tet, 2 sub-tets
        per polygon edge of each of the two cells of a face)."""
        est = self.afe.estimate_bytes(req.mesh, req.N, req.params or self.afe.Params())
        npn = (req.N + 1) * (req.N + 2) * (req.N + 3) // 6
        nodes = npn * 2 * int(np.diff(req.mesh["face_ptr"]).sum())
        return est + 13 * 8 * nodes

    def setup(self, req: Request):
        torch = self.torch
        if not hasattr(self.local, "stream"):
            self.local.stream = torch.cuda.Stream()
        st = self.local.stream
        with torch.cuda.stream(st):
            cd = self.afe.CellData(req.mesh, req.N, req.params or self.afe.Params(), stream=st)
            x = cd.dof_coords(stream=st).cpu().numpy()
            prim = torch.tensor(req.field(np.mod(x.T, req.mesh["box"])).T.copy(), device="cuda")
            u = cd.prim_to_cons(prim, stream=st)
            st.synchronize()
        return cd, u

    def attach(self, handle, req: Request) -> int:
        cd, u = handle
        return self.batch.attach(cd, u, req.cfl)

    def step(self) -> dict:
        reps = self.batch.step(stream=self.step_stream, check=False)
        return {slot: (r.status, r.iters_mean) for slot, r in reps.items()}

    def release(self, handle, keep_state: bool):
        cd, u = handle
        self.batch.detach(cd)
        state = u.cpu().numpy() if keep_state else None
        cd.close()
        return state, cd.ndof

    def discard(self, handle):
        """Frees a set-up request that never joined the batch."""
        handle[0].close()

    def ndof(self, handle) -> int:
        return handle[0].ndof


class Server:
    """Continuous-batching request loop with device-memory admission."""

    def __init__(self, backend, hbm_budget: int, max_active: int = 64, keep_states: bool = False,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 setup_workers: int = 2):
        self.be = backend
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.keep_states = keep_states
        self.clock = clock
        self.sleep = sleep
        self.setup_workers = setup_workers
        self.peak_bytes = 0
        self.peak_active = 0
        self.steps_run = 0

    def run(self, requests: list[Request]) -> list[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results = {r.rid: Result(r.rid, r.arrival) for r in reqs}
        waiting = collections.deque(reqs)
        setting_up = {}   # future -> request
        active = {}       # slot -> (request, handle, result)
        used = 0
        est = {}
        t0 = self.clock()
        pool = cf.ThreadPoolExecutor(max_workers=self.setup_workers)
        try:
            while waiting or setting_up or active:
                now = self.clock() - t0
                # admission in arrival order (a request that can never fit is rejected)
                while waiting and waiting[0].arrival <= now and len(active) + len(setting_up) < self.max_active:
                    r = waiting[0]
                    if r.rid not in est:
                        est[r.rid] = self.be.estimate(r)
                    if est[r.rid] > self.budget:
                        waiting.popleft()
                        res = results[r.rid]
                        res.admitted = res.ready = res.done = now
                        res.status = "AFE_E_HBM_BUDGET"
                        continue
                    if used + est[r.rid] > self.budget:
                        break
                    waiting.popleft()
                    used += est[r.rid]
                    self.peak_bytes = max(self.peak_bytes, used)
                    results[r.rid].admitted = now
                    results[r.rid].bytes = est[r.rid]
                    setting_up[pool.submit(self.be.setup, r)] = r
                # set-ups that finished join at this step boundary
                for f in [f for f in setting_up if f.done()]:
                    r = setting_up.pop(f)
                    res = results[r.rid]
                    res.ready = self.clock() - t0
                    try:
                        handle = f.result()
                    except Exception as e:  # noqa: BLE001 - a failed set-up fails its request only
                        res.status = getattr(e, "name", type(e).__name__)
                        res.done = res.ready
                        used -= est[r.rid]
                        continue
                    res.ndof = self.be.ndof(handle)
                    try:
                        slot = self.be.attach(handle, r)
                    except Exception as e:  # noqa: BLE001 - a refused join fails its request only
                        res.status = getattr(e, "name", type(e).__name__)
                        res.done = res.ready
                        self.be.discard(handle)
                        used -= est[r.rid]
                        continue
                    active[slot] = (r, handle, res)
                if not active:
                    nxt = [waiting[0].arrival - (self.clock() - t0)] if waiting else []
                    wait = min([0.002] + [t for t in nxt if t > 0])
                    if setting_up:
                        cf.wait(list(setting_up), timeout=wait, return_when=cf.FIRST_COMPLETED)
                    elif wait > 0:
                        self.sleep(wait)
                    continue
                self.peak_active = max(self.peak_active, len(active))
                reps = self.be.step()
                self.steps_run += 1
                now = self.clock() - t0
                for slot, (status, iters) in reps.items():
                    r, handle, res = active[slot]
                    res.steps_done += 1
                    res.iters_mean.append(iters)
                    if status != "AFE_OK":
                        res.status = status
                    if res.steps_done >= r.steps or status != "AFE_OK":
                        res.done = now
                        res.state, _ = self.be.release(handle, self.keep_states)
                        used -= est[r.rid]
                        del active[slot]
        finally:
            pool.shutdown(wait=True)
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(results: list[Result], makespan: float | None = None) -> dict:
    """p50/p99 latency (and its parts) over completed requests, aggregate
    DOF-updates/s = sum(5 ndof steps) / (last completion - first arrival)."""
    ok = [r for r in results if r.status == "AFE_OK"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    span = makespan if makespan is not None else (max(r.done for r in results) - min(r.arrival for r in results))
    work = sum(5 * r.ndof * r.steps_done for r in ok)

    def pct(a, q):
        return float(np.percentile(a, q)) if len(a) else float("nan")
    return {
        "requests": len(results), "completed": len(ok),
        "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
        "queue_p50_s": pct(np.array([r.queue for r in ok]), 50),
        "setup_p50_s": pct(np.array([r.setup for r in ok]), 50),
        "solve_p50_s": pct(np.array([r.solve for r in ok]), 50),
        "dof_updates_per_s": work / span if span > 0 else float("nan"),
        "makespan_s": span,
    }
