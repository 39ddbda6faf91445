"""Continuous-batching server for parametric sweeps of the clap & fling solve.

The paper studies one flow at many parameter points (Re, J and f varied,
Sec. 3.3-3.5).  Served here, each point is a request that arrives at some
time; the server keeps every admitted solve's lattice resident on the
device, admits waiting requests in arrival order whenever their workspace
fits in the HBM budget (and a batch slot is free), and advances all admitted
solves together with ``ibmlbm_step_batch``: every stage of a time step is
one grouped launch over all of them, so a newly admitted solve shares the
device with the ones already running from its first step on.  A solve is
retired (its force history read, its workspace released) as soon as its
last step has run, which frees memory and a slot for the next request.

Each solve runs the same kernels with the same arguments as when stepped
alone, so its results do not depend on what else is in the batch.

Latency of a request = time its result is available - its arrival time.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import time
from typing import Callable, List, Optional, Union

import numpy as np

from .solver import Solver, step_batch, workspace_bytes

MAX_BATCH = 64       # solves per grouped launch (the library's limit)
PREFETCH_BYTES = 4 << 30   # host memory for initial fields made ahead of admission


@dataclasses.dataclass
class SweepRequest:
    """One solve: a complete box and foil description (tau, inlet velocity,
    reference velocity and periods filled in), the number of steps, the
    arrival time in seconds from the start of the run and the initial
    velocity field (an array, or a callable that makes it at admission)."""
    rid: int
    box: dict
    wings: list
    steps: int
    arrival: float = 0.0
    u0: Union[None, np.ndarray, Callable[[], np.ndarray]] = None
    storage: str = "fp32"


@dataclasses.dataclass
class SweepResult:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    cells: int
    forces: Optional[np.ndarray]        # [steps][n_wings][8]
    error: Optional[str] = None

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclasses.dataclass
class _Active:
    req: SweepRequest
    solver: Solver
    admitted: float
    fp: int = 0
    done: int = 0


class GpuBackend:
    """Solves on one ROCm device through libibmlbm.  A new solve is set up
    (workspace, markers, initial state) on a side stream, so the batch
    already running on the compute stream keeps the device busy meanwhile,
    and then joins the compute stream.  The solves admitted together are set
    up on several host threads (the library keeps no shared state between
    handles, and its host-side geometry is most of a set-up)."""

    parallel_create = True

    def __init__(self, device="cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the sweep server needs a ROCm GPU")
        self.device = torch.device(device)
        self.torch = torch
        self.compute = torch.cuda.current_stream(self.device)
        self.side = torch.cuda.Stream(self.device)
        self._fp = {}   # footprints by request id, handed on to create()

    def free_bytes(self):
        return self.torch.cuda.mem_get_info(self.device)[0]

    def footprint(self, req: SweepRequest) -> int:
        fp = workspace_bytes(req.box, req.wings, req.storage, history_steps=max(req.steps, 1))
        self._fp[req.rid] = fp
        return fp

    def create(self, req: SweepRequest, u0=None):
        s = Solver(req.box, req.wings, storage=req.storage, history_steps=max(req.steps, 1),
                   device=self.device, stream=self.side, nbytes=self._fp.pop(req.rid, None) or None)
        if u0 is None:
            u0 = req.u0() if callable(req.u0) else req.u0
        s.init_fields(u=u0)
        s.set_stream(self.compute)
        return s

    def step(self, solvers, n):
        step_batch(solvers, n)

    def release(self, solver):
        solver.close()
        solver.ws = None


class SweepServer:
    """Request loop over one device.

    hbm_budget: bytes of device memory the resident solves may hold (None =
        90% of the free device memory at construction).
    chunk: steps enqueued per round of the loop; a round ends early when a
        solve completes, so results are never held back by a chunk.
    max_batch: solves stepped together (at most 64).
    backend: where solves live (default: the GPU through libibmlbm).
    """

    def __init__(self, hbm_budget=None, chunk=50, max_batch=MAX_BATCH, device="cuda:0",
                 backend=None):
        self.backend = backend if backend is not None else GpuBackend(device)
        if hbm_budget is None:
            hbm_budget = int(0.9 * self.backend.free_bytes())
        self.budget = int(hbm_budget)
        self.chunk = max(1, int(chunk))
        self.max_batch = max(1, min(int(max_batch), MAX_BATCH))
        self.batch_sizes: List[int] = []   # solves per grouped round, for reporting
        self.peak_bytes = 0

    def footprint(self, req: SweepRequest) -> int:
        return self.backend.footprint(req)

    def run(self, requests, log: Optional[Callable[[str], None]] = None):
        """Serve `requests` (arrival times relative to now) to completion;
        returns the results in request order."""
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        pool = concurrent.futures.ThreadPoolExecutor(max_workers=4)
        makers = (concurrent.futures.ThreadPoolExecutor(max_workers=4)
                  if getattr(self.backend, "parallel_create", False) else None)
        prepared = {}

        def prefetch():
            # make the initial fields of the waiting requests that the next
            # admissions can take (up to a batch, within PREFETCH_BYTES of
            # host memory) on host threads while the device works, so that
            # admitting a batch does not wait for them
            held = 0
            for r in list(waiting)[:self.max_batch]:
                if not callable(r.u0):
                    continue
                held += 24 * r.box["nx"] * r.box["ny"] * r.box["nz"]   # 3 FP64 components
                if held > PREFETCH_BYTES:
                    break
                if r.rid not in prepared:
                    prepared[r.rid] = pool.submit(r.u0)

        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque = collections.deque()
        active: List[_Active] = []
        results = {}
        used = 0
        fp_cache = {}
        def admit():
            # admission, in arrival order: a request waits for memory rather
            # than being overtaken by a smaller one
            nonlocal used
            chosen = []
            while waiting and len(active) + len(chosen) < self.max_batch:
                r = waiting[0]
                fp = fp_cache.get(r.rid)
                if fp is None:
                    fp = fp_cache[r.rid] = self.footprint(r)
                if fp == 0 or fp > self.budget:
                    waiting.popleft()
                    prepared.pop(r.rid, None)
                    why = "invalid solve description" if fp == 0 else "larger than the HBM budget"
                    t = now()
                    results[r.rid] = SweepResult(r.rid, r.arrival, t, t, 0, 0, None, why)
                    continue
                if used + fp > self.budget:
                    break
                waiting.popleft()
                used += fp
                self.peak_bytes = max(self.peak_bytes, used)
                chosen.append((r, fp, prepared.pop(r.rid, None)))
            if not chosen:
                return

            def make(item):
                r, _, fut = item
                return self.backend.create(r, fut.result() if fut is not None else None)

            # the solves admitted together are set up at once where the
            # backend allows it, and join the batch in admission order
            made = list(makers.map(make, chosen)) if makers is not None and len(chosen) > 1 else \
                [make(c) for c in chosen]
            for (r, fp, _), s in zip(chosen, made):
                active.append(_Active(r, s, now(), fp=fp))
                if log:
                    log(f"admit {r.rid} at {now():.3f}s ({len(active)} active, {used / 2**20:.0f} MiB)")

        while pending or waiting or active:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            prefetch()
            # one round: the next chunk of the running solves is enqueued
            # first, so that setting up newly admitted solves (on the side
            # stream) overlaps it; those join from the next round on
            stepping = list(active)
            k = min(self.chunk, min(a.req.steps - a.done for a in stepping)) if stepping else 0
            if k > 0:
                self.backend.step([a.solver for a in stepping], k)
                self.batch_sizes.append(len(stepping))
                for a in stepping:
                    a.done += k
            admit()
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - now()))
                continue
            keep = []
            for a in active:
                if a.done < a.req.steps:
                    keep.append(a)
                    continue
                f = a.solver.forces(0, a.req.steps) if a.req.wings else None   # synchronises
                cells = a.req.box["nx"] * a.req.box["ny"] * a.req.box["nz"]
                results[a.req.rid] = SweepResult(a.req.rid, a.req.arrival, a.admitted, now(),
                                                 a.req.steps, cells, f)
                used -= a.fp
                self.backend.release(a.solver)
                if log:
                    log(f"done {a.req.rid} at {now():.3f}s")
            active = keep
        pool.shutdown(wait=True)
        if makers is not None:
            makers.shutdown(wait=True)
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(results):
    """p50 / p99 latency (s), aggregate MLUPS over the run's span, counts."""
    ok = [r for r in results if r.error is None]
    if not ok:
        return dict(requests=len(results), completed=0)
    lat = np.array([r.latency for r in ok])
    start = min(r.arrival for r in ok)
    end = max(r.finished for r in ok)
    updates = sum(r.cells * r.steps for r in ok)
    return dict(requests=len(results), completed=len(ok),
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), span_s=float(end - start),
                mlups=float(updates / max(end - start, 1e-9) / 1e6))
