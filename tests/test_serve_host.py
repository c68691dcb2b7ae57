"""Host logic of the serving loop with a fake backend and a virtual clock (no
GPU): admission in arrival order under the device-memory budget and the slot
limit, continuous batching (arrivals join running batches at step
boundaries), release after the last step or a failed step, rejection of a
request that can never fit, latency bookkeeping."""
import threading
import time

import numpy as np
import pytest

from paper_2605_00619_amd.serve import Request, Server, summarize


class Clock:
    def __init__(self):
        self.t = 0.0
        self.lock = threading.Lock()

    def __call__(self):
        with self.lock:
            return self.t

    def advance(self, dt):
        with self.lock:
            self.t += dt


class _Refused(Exception):
    name = "AFE_E_ARG"


class FakeBackend:
    """Each request's mesh dict carries its byte size, DOF count, the step at
    which it fails (if any); a step takes 10 ms of virtual time."""

    def __init__(self, clock, budget):
        self.clock = clock
        self.budget = budget
        self.live = {}       # slot -> (rid, bytes)
        self.next_slot = 0
        self.log = []        # (time, event, rid)
        self.max_live_bytes = 0
        self.steps = {}      # rid -> steps taken
        self.batch_sizes = []

    def estimate(self, req):
        return req.mesh["bytes"]

    def setup(self, req):
        return req

    def ndof(self, req):
        return req.mesh["ndof"]

    def attach(self, req, _):
        if req.mesh.get("refuse"):
            raise _Refused()
        slot = self.next_slot
        self.next_slot += 1
        self.live[slot] = (req, req.mesh["bytes"])
        self.steps[req.rid] = 0
        self.max_live_bytes = max(self.max_live_bytes, sum(b for _, b in self.live.values()))
        assert self.max_live_bytes <= self.budget
        self.log.append((self.clock(), "join", req.rid))
        return slot

    def step(self):
        time.sleep(0.001)  # a real step takes time; the set-up thread runs meanwhile
        self.clock.advance(0.010)
        self.batch_sizes.append(len(self.live))
        out = {}
        for slot, (req, _) in self.live.items():
            self.steps[req.rid] += 1
            fail = req.mesh.get("fail_at") == self.steps[req.rid]
            out[slot] = ("AFE_E_POSITIVITY" if fail else "AFE_OK", 3.0)
        return out

    def release(self, req, keep):
        slot = [s for s, (r, _) in self.live.items() if r is req][0]
        del self.live[slot]
        self.log.append((self.clock(), "leave", req.rid))
        return None, req.mesh["ndof"]

    def discard(self, req):
        self.log.append((self.clock(), "discard", req.rid))


def _req(rid, arrival, nbytes, steps, ndof=100, fail_at=None, refuse=False):
    return Request(rid, arrival, dict(bytes=nbytes, ndof=ndof, fail_at=fail_at, refuse=refuse), 2, steps, 0.1,
                   lambda x: x)


def _serve(reqs, budget, max_active=64):
    clock = Clock()
    be = FakeBackend(clock, budget)
    srv = Server(be, budget, max_active=max_active, clock=clock, sleep=clock.advance)
    return srv.run(reqs), be, srv


def test_continuous_batching_under_budget():
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(1 / 50.0, size=40))
    sizes = rng.integers(1, 6, size=40) * 10
    steps = rng.integers(2, 12, size=40)
    reqs = [_req(i, float(a), int(b), int(s)) for i, (a, b, s) in enumerate(zip(arrivals, sizes, steps))]
    res, be, srv = _serve(reqs, budget=100)
    assert all(r.status == "AFE_OK" for r in res)
    assert [r.steps_done for r in res] == [int(s) for s in steps]
    assert be.max_live_bytes <= 100 and srv.peak_bytes <= 100
    # admission in arrival order
    adm = [r.admitted for r in sorted(res, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    # some requests waited for memory, and batches mixed requests of different ages
    assert max(r.queue for r in res) > 0.0
    joins = {rid: t for t, ev, rid in be.log if ev == "join"}
    leaves = {rid: t for t, ev, rid in be.log if ev == "leave"}
    overlap = sum(1 for a in joins for b in joins if a != b and joins[a] < joins[b] < leaves[a])
    assert overlap > 0
    assert max(be.batch_sizes) > 1
    for r in res:
        assert r.arrival <= r.admitted <= r.ready <= r.done
        assert abs(r.latency - (r.queue + r.setup + r.solve)) < 1e-12
    s = summarize(res)
    assert s["completed"] == 40 and s["latency_p50_s"] <= s["latency_p99_s"]
    assert s["dof_updates_per_s"] > 0


def test_slot_limit_and_rejection_and_failure():
    reqs = [_req(0, 0.0, 10, 5), _req(1, 0.0, 10, 5), _req(2, 0.0, 10, 5),
            _req(3, 0.001, 500, 3),                 # never fits: rejected
            _req(4, 0.002, 10, 6, fail_at=2)]       # fails at its second step
    res, be, srv = _serve(reqs, budget=100, max_active=2)
    assert max(be.batch_sizes) <= 2
    assert res[3].status == "AFE_E_HBM_BUDGET" and res[3].steps_done == 0
    assert res[4].status == "AFE_E_POSITIVITY" and res[4].steps_done == 2
    assert all(res[i].status == "AFE_OK" and res[i].steps_done == 5 for i in range(3))
    assert len(be.live) == 0
    # the third request waited for a slot, not for memory
    assert res[2].queue > 0.0


def test_refused_join_fails_only_its_request():
    """A set-up request the batch refuses to join (a bounded mesh, which
    batches do not take) is retired with the refusal's status, freed, and its
    memory returned; the other requests run to completion."""
    reqs = [_req(0, 0.0, 40, 4), _req(1, 0.0, 50, 4, refuse=True), _req(2, 0.001, 50, 4)]
    res, be, srv = _serve(reqs, budget=100)
    assert res[1].status == "AFE_E_ARG" and res[1].steps_done == 0
    assert res[1].done == res[1].ready
    assert [r.status for r in (res[0], res[2])] == ["AFE_OK", "AFE_OK"]
    assert [r.steps_done for r in (res[0], res[2])] == [4, 4]
    assert [rid for _, ev, rid in be.log if ev == "discard"] == [1]
    assert len(be.live) == 0


class _FailingLib:
    """Stand-in for libafe whose batch step fails before it fills any report
    (as a HIP launch or allocation failure does)."""

    def afe_batch_step(self, h, reps, n, stream):
        return -7

    def afe_last_error(self):
        return b"launch failed"


def test_call_failure_marks_every_served_request_failed(monkeypatch):
    """A batch step that fails as a call (AFE_E_HIP) leaves the reports
    unfilled; the binding gives every member the call's status, so the server
    retires the requests as failed instead of counting a step that never ran."""
    import types

    from paper_2605_00619_amd import afe
    from paper_2605_00619_amd.serve import GpuBackend

    monkeypatch.setattr(afe, "_lib", _FailingLib())
    batch = object.__new__(afe.Batch)
    batch._h = None
    batch._members = {}
    reps = batch.step(stream=0, check=False)
    assert reps == {}

    class Backend(FakeBackend):
        def attach(self, req, _):
            slot = super().attach(req, _)
            batch._members[slot] = (None, None)
            return slot

        def step(self):
            return GpuBackend.step(self)

        def release(self, req, keep):
            slot = [s for s, (r, _) in self.live.items() if r is req][0]
            del batch._members[slot]
            return super().release(req, keep)

    clock = Clock()
    be = Backend(clock, 100)
    be.batch = batch
    be.step_stream = types.SimpleNamespace(cuda_stream=0)
    res = Server(be, 100, clock=clock, sleep=clock.advance).run([_req(0, 0.0, 10, 5), _req(1, 0.0, 10, 5)])
    assert [r.status for r in res] == ["AFE_E_HIP", "AFE_E_HIP"]
    assert [r.steps_done for r in res] == [1, 1]
    assert summarize(res)["completed"] == 0
    with pytest.raises(afe.AfeError):
        batch.step(stream=0, check=True)
