"""Scheduling policy of the sweep server on the host, with a stand-in
backend (no GPU): admission in arrival order under the HBM budget and the
batch limit, late arrivals joining running batches, rejection of requests
that can never fit, retirement as soon as a solve's last step has run, and
the latency summary."""
import time

import numpy as np
import pytest

from paper_2102_01305_amd.serve import SweepRequest, SweepServer, summarize


class FakeSolver:
    def __init__(self, req):
        self.req = req
        self.steps = 0
        self.released = False

    def forces(self, first, count):
        return np.zeros((count, len(self.req.wings), 8))


class FakeBackend:
    """Footprint = box['bytes']; each grouped round of k steps takes k ms."""

    def __init__(self, free=1 << 40, step_s=1e-3):
        self.free = free
        self.step_s = step_s
        self.rounds = []          # rids stepped together per round
        self.admitted = []        # admission order

    def free_bytes(self):
        return self.free

    def footprint(self, req):
        return req.box["bytes"]

    def create(self, req, u0=None):
        self.admitted.append(req.rid)
        self.u0s = getattr(self, "u0s", []) + [u0]
        return FakeSolver(req)

    def step(self, solvers, n):
        assert all(not s.released for s in solvers)
        self.rounds.append(sorted(s.req.rid for s in solvers))
        for s in solvers:
            s.steps += n
        time.sleep(self.step_s * n)

    def release(self, solver):
        assert solver.steps == solver.req.steps, "retired before its last step"
        solver.released = True


def _req(rid, nbytes, steps, arrival=0.0):
    return SweepRequest(rid=rid, box=dict(nx=4, ny=4, nz=4, bytes=nbytes), wings=[{}],
                        steps=steps, arrival=arrival)


def test_admission_respects_budget_and_arrival_order():
    be = FakeBackend()
    srv = SweepServer(hbm_budget=6, chunk=5, backend=be)
    reqs = [_req(0, 3, 20), _req(1, 3, 40), _req(2, 3, 10), _req(3, 1, 10), _req(4, 1, 10)]
    res = srv.run(reqs)
    assert [r.rid for r in res] == [0, 1, 2, 3, 4]
    assert all(r.error is None for r in res)
    assert be.admitted == [0, 1, 2, 3, 4]            # no overtaking
    assert srv.peak_bytes <= 6
    # at most two 3-byte solves resident at once; 3 waits for 2 to be admitted
    for rnd in be.rounds:
        assert sum(3 if rid < 3 else 1 for rid in rnd) <= 6
    # request 2 starts only after request 0 retires (memory)
    first_round_with_2 = next(i for i, r in enumerate(be.rounds) if 2 in r)
    assert all(0 not in r for r in be.rounds[first_round_with_2:])


def test_batch_limit_and_late_arrivals_join_running_batches():
    be = FakeBackend(step_s=2e-3)
    srv = SweepServer(hbm_budget=100, chunk=4, max_batch=3, backend=be)
    reqs = [_req(i, 1, 40) for i in range(3)] + [_req(3, 1, 8, arrival=0.03), _req(4, 1, 8, arrival=0.03)]
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert max(len(r) for r in be.rounds) <= 3
    # the late requests arrive while three solves fill the batch: they wait
    # for a slot, which the first retirement frees
    assert max(srv.batch_sizes) == 3
    late = [r for r in res if r.rid >= 3]
    early_done = min(r.finished for r in res if r.rid < 3)
    assert all(r.admitted >= early_done - 1e-9 for r in late)


def test_late_arrival_joins_a_running_solve():
    be = FakeBackend(step_s=2e-3)
    srv = SweepServer(hbm_budget=100, chunk=5, backend=be)
    res = srv.run([_req(0, 1, 60), _req(1, 1, 10, arrival=0.02)])
    both = [r for r in be.rounds if r == [0, 1]]
    assert both, be.rounds
    r0, r1 = res
    assert r1.admitted < r0.finished and r1.finished < r0.finished


def test_oversized_request_is_rejected_others_served():
    be = FakeBackend()
    srv = SweepServer(hbm_budget=10, chunk=10, backend=be)
    res = srv.run([_req(0, 11, 10), _req(1, 5, 10)])
    assert res[0].error and "budget" in res[0].error
    assert res[1].error is None and res[1].steps == 10


def test_summary_percentiles_and_rate():
    be = FakeBackend()
    srv = SweepServer(hbm_budget=100, chunk=10, backend=be)
    res = srv.run([_req(i, 1, 10 * (i + 1)) for i in range(5)])
    s = summarize(res)
    lat = np.array([r.latency for r in res])
    assert s["completed"] == 5
    assert s["p50_s"] == pytest.approx(float(np.percentile(lat, 50)))
    assert s["p99_s"] == pytest.approx(float(np.percentile(lat, 99)))
    assert s["mlups"] > 0


def test_initial_fields_made_ahead_within_the_host_bound(monkeypatch):
    """The fields of waiting requests are made on host threads before their
    admission, as far as PREFETCH_BYTES of host memory allows; a request past
    that bound is handed no field (its backend makes it at admission)."""
    from paper_2102_01305_amd import serve

    made = []

    def field(rid):
        def make():
            made.append(rid)
            return np.full((3, 4, 4, 4), float(rid))
        return make

    # room for two 4 x 4 x 4 fields of 3 FP64 components
    monkeypatch.setattr(serve, "PREFETCH_BYTES", 2 * 24 * 64)
    be = FakeBackend()
    srv = SweepServer(hbm_budget=100, chunk=10, max_batch=6, backend=be)
    reqs = [SweepRequest(rid=i, box=dict(nx=4, ny=4, nz=4, bytes=1), wings=[{}], steps=10, u0=field(i))
            for i in range(6)]
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert be.admitted == list(range(6))
    got = [None if u is None else int(u[0, 0, 0, 0]) for u in be.u0s]
    assert got == [0, 1, None, None, None, None]
    assert sorted(made) == [0, 1]


def test_parallel_set_up_keeps_the_schedule():
    """A backend that sets up the solves admitted together on several host
    threads (parallel_create) gets the same batches, in the same rounds, as
    one that sets them up one by one, whatever order the threads finish in."""
    import random

    class Slow(FakeBackend):
        def create(self, req, u0=None):
            time.sleep(random.Random(req.rid).uniform(0.0, 2e-3))
            return super().create(req, u0)

    class Parallel(Slow):
        parallel_create = True

    reqs = [_req(i, 1 + i % 3, 10 + 5 * (i % 4)) for i in range(10)]
    runs = []
    for cls in (Slow, Parallel):
        be = cls(step_s=2e-4)
        srv = SweepServer(hbm_budget=8, chunk=5, max_batch=4, backend=be)
        res = srv.run(reqs)
        assert all(r.error is None for r in res)
        runs.append((be.rounds, sorted(be.admitted)))
    assert runs[0][1] == runs[1][1] == list(range(10))
    assert runs[0][0] == runs[1][0]
