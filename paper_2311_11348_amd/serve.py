"""Continuous-batching service for independent shallow-water solves.

Requests arrive over time (each: a mesh size, an order, a step count and a
forcing kind).  Host threads prepare each request's context (mesh upload,
bathymetry, initial state) once it has arrived and the prepared contexts'
footprints fit the staging budget (a prepared context holds device memory
until it is admitted); the scheduler admits prepared requests into the
resident batch while their device footprint fits the budget (the batch
itself refuses any admission that would take its own device memory beyond
the budget), advances every resident instance together (one step graph per
tick, each instance at its own time step and step budget), retires finished
instances (state copied back to the host) and admits the next ones at every
tick boundary.  Latency is measured from arrival to the completed copy of the
result.  A request that fails (invalid input, non-finite value or
non-positive depth during the run) is reported failed alone; the others are
unaffected.

The scheduler is written against a small executor interface so that its
logic (admission, FIFO order, latency accounting, failure isolation) can be
tested without a GPU.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import inputs as I


@dataclass
class Request:
    rid: int
    spec: I.Request           # arrival time (s after the start), seed, size, order, steps, kind
    poisoned: bool = False    # test hook: an initial state with negative depth everywhere

    @property
    def arrival(self) -> float:
        return self.spec.arrival

    @property
    def elements(self) -> int:
        n = I.instance_mesh_n(self.spec.n_elements_target)
        return 2 * n * n


@dataclass
class Result:
    rid: int
    ok: bool
    arrival: float
    admitted: float
    done: float
    dof_updates: float
    state: Optional[np.ndarray] = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def requests_from_trace(trace: List[I.Request]) -> List[Request]:
    return [Request(rid=i, spec=r) for i, r in enumerate(trace)]


class Executor:
    """What the scheduler needs from the device side."""

    def footprint(self, req: Request) -> int: ...
    def budget(self) -> int: ...
    def prepare(self, req: Request): ...          # host thread; returns an opaque handle
    def admit(self, handle) -> int: ...           # returns a slot
    def tick(self, nsteps: int) -> None: ...
    def poll(self) -> List: ...                   # [(slot, failed)]
    def retire(self, slot: int, failed: bool): ...  # returns (state or None, dof_updates)
    def discard(self, handle) -> None: ...        # a prepared request that is never admitted


def _initial_state(ctx, prob, req, init_state):
    """Set a request's initial state: its analytic initial condition projected
    on the device, or the coefficients init_state(problem) returns (callers
    that bring their own projection), or a dry state for a poisoned request."""
    if req.poisoned:
        c = np.zeros((prob.mesh.ne, 3, I.K_OF_P[req.spec.p]))
        c[:, 0, 0] = -5000.0 * np.sqrt(prob.mesh.areas())   # every element dry
        ctx.set_state(c)
    elif init_state is not None:
        ctx.set_state(init_state(prob))
    else:
        ctx.set_state_fn(prob.ic)


class GpuExecutor(Executor):
    def __init__(self, precision: int, budget_bytes: int, max_instances: int = 1024, stream=None,
                 keep_state: bool = True, init_state: Optional[Callable] = None):
        from . import swe
        self.swe = swe
        self.precision = precision
        self.batch = swe.Batch(precision=precision, budget_bytes=budget_bytes, max_instances=max_instances,
                               stream=stream)
        self._budget = budget_bytes
        self.keep_state = keep_state
        self.init_state = init_state
        self.slots: Dict[int, tuple] = {}

    def footprint(self, req):
        return self.swe.swe_footprint_bytes(req.elements, req.spec.p, self.precision)

    def budget(self):
        return self._budget

    def prepare(self, req):
        prob = I.request_problem(req.spec)
        ctx = self.swe.context_for(prob, precision=self.precision)
        _initial_state(ctx, prob, req, self.init_state)
        return ctx, prob.dt(), req.spec.steps, 3 * I.K_OF_P[req.spec.p] * prob.mesh.ne

    def admit(self, handle):
        ctx, dt, steps, dof = handle
        slot = self.batch.admit(ctx, steps, dt)
        self.slots[slot] = (ctx, dof * 2 * steps)
        return slot

    def tick(self, nsteps):
        self.batch.tick(nsteps)

    def poll(self):
        return self.batch.poll()

    def retire(self, slot, failed):
        ctx, dof = self.slots.pop(slot)
        self.batch.retire(slot)
        state = None
        if not failed and self.keep_state:
            state, _ = ctx.state()
        ctx.close()
        return state, dof

    def discard(self, handle):
        handle[0].close()

    def close(self):
        self.batch.close()


class PlainExecutor(Executor):
    """The plain solver: one request on the GPU at a time, unbatched, each
    stage one ordinary launch over that request's mesh (FIFO queue).  Each
    context runs on its own streams, so preparing the next requests does not
    queue behind (or ahead of) the running one."""

    def __init__(self, precision: int, budget_bytes: int = 64 << 30, keep_state: bool = True,
                 init_state: Optional[Callable] = None):
        from . import swe
        self.swe = swe
        self.precision = precision
        self._budget = budget_bytes
        self.keep_state = keep_state
        self.init_state = init_state
        self.cur: Dict[int, list] = {}
        self.next_slot = 0

    def footprint(self, req):
        return self.swe.swe_footprint_bytes(req.elements, req.spec.p, self.precision)

    def budget(self):
        return self._budget

    def prepare(self, req):
        prob = I.request_problem(req.spec)
        ctx = self.swe.context_for(prob, precision=self.precision)
        _initial_state(ctx, prob, req, self.init_state)
        return ctx, prob.dt(), req.spec.steps, 3 * I.K_OF_P[req.spec.p] * prob.mesh.ne

    def admit(self, handle):
        if self.cur:
            raise RuntimeError("the plain solver holds one request at a time")
        ctx, dt, steps, dof = handle
        s = self.next_slot
        self.next_slot += 1
        self.cur[s] = [ctx, dt, steps, dof * 2 * steps, False]
        return s

    def tick(self, nsteps):
        for s, m in self.cur.items():
            n = min(nsteps, m[2])
            try:
                m[0].step(n, m[1])
                m[0].sync()
            except self.swe.SweError:
                m[4] = True
            m[2] -= n

    def poll(self):
        return [(s, m[4]) for s, m in self.cur.items() if m[2] <= 0 or m[4]]

    def retire(self, slot, failed):
        ctx, _, _, dof, _ = self.cur.pop(slot)
        state = None
        if not failed and self.keep_state:
            state, _ = ctx.state()
        ctx.close()
        return state, dof

    def discard(self, handle):
        handle[0].close()

    def close(self):
        pass


@dataclass
class ServeStats:
    results: List[Result] = field(default_factory=list)
    wall: float = 0.0
    max_used: int = 0
    max_staged: int = 0
    ticks: int = 0

    def summary(self) -> dict:
        ok = [r for r in self.results if r.ok]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        dof = sum(r.dof_updates for r in ok)
        return {"requests": len(self.results), "completed": len(ok),
                "failed": len(self.results) - len(ok),
                "solves_per_s": len(ok) / self.wall if self.wall > 0 else 0.0,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "dof_updates_per_s": dof / self.wall if self.wall > 0 else 0.0,
                "wall_s": self.wall, "max_resident_bytes": self.max_used, "max_staged_bytes": self.max_staged,
                "ticks": self.ticks}


def serve(requests: List[Request], ex: Executor, tick_steps: int = 50, prep_threads: int = 8,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          on_tick: Optional[Callable[[float, int], None]] = None,
          stage_budget: Optional[int] = None) -> ServeStats:
    """Run the request trace to completion and return per-request results.

    stage_budget bounds the summed footprints of the requests being prepared
    or prepared and waiting for admission (their contexts hold device memory
    beside the resident batch); default a quarter of the executor's budget.
    One request is always let through, so any request can make progress."""
    stats = ServeStats()
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    preparing: deque = deque()                 # (request, future, footprint) in arrival order
    resident: Dict[int, tuple] = {}            # slot -> (request, admitted time, footprint)
    used = staged = 0
    stage_cap = ex.budget() // 4 if stage_budget is None else stage_budget
    t0 = clock()
    pool = ThreadPoolExecutor(max_workers=prep_threads)
    try:
        while pending or preparing or resident:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                fp = ex.footprint(pending[0])
                if preparing and staged + fp > stage_cap:
                    break                       # wait until admissions free staging room
                r = pending.popleft()
                preparing.append((r, pool.submit(ex.prepare, r), fp))
                staged += fp
                stats.max_staged = max(stats.max_staged, staged)
            # admission at the tick boundary, FIFO: the head waits until it fits
            while preparing and preparing[0][1].done():
                r, fut, fp = preparing[0]
                err = fut.exception()
                if err is not None:
                    preparing.popleft()
                    staged -= fp
                    stats.results.append(Result(r.rid, False, r.arrival, now, clock() - t0, 0.0, error=str(err)))
                    continue
                if used + fp > ex.budget():
                    if not resident:          # can never fit
                        preparing.popleft()
                        staged -= fp
                        ex.discard(fut.result())
                        stats.results.append(Result(r.rid, False, r.arrival, now, clock() - t0, 0.0,
                                                    error="footprint exceeds the budget"))
                        continue
                    break
                try:
                    slot = ex.admit(fut.result())
                except Exception as e:          # no free slot or no room in the pools: retry after a retirement
                    if not resident:
                        preparing.popleft()
                        staged -= fp
                        ex.discard(fut.result())
                        stats.results.append(Result(r.rid, False, r.arrival, now, clock() - t0, 0.0, error=str(e)))
                        continue
                    break
                preparing.popleft()
                staged -= fp
                resident[slot] = (r, clock() - t0, fp)
                used += fp
                stats.max_used = max(stats.max_used, used)
            if resident:
                ex.tick(tick_steps)
                stats.ticks += 1
                for slot, failed in ex.poll():
                    r, adm, fp = resident.pop(slot)
                    used -= fp
                    state, dof = ex.retire(slot, failed)
                    stats.results.append(Result(r.rid, not failed, r.arrival, adm, clock() - t0,
                                                dof if not failed else 0.0, state=state,
                                                error="non-finite value or non-positive depth" if failed else ""))
                if on_tick:
                    on_tick(clock() - t0, len(resident))
            else:
                nxt = pending[0].arrival if pending else None
                if preparing:
                    sleep(0.001)
                elif nxt is not None:
                    sleep(max(0.0, min(0.05, nxt - (clock() - t0))))
        stats.wall = clock() - t0
    finally:
        pool.shutdown(wait=True)
    stats.results.sort(key=lambda r: r.rid)
    return stats


class FakeExecutor(Executor):
    """Timing model for CPU tests: a tick costs step_time * nsteps; prepare can fail."""

    def __init__(self, budget_bytes: int, bytes_per_element: int = 100, step_time: float = 0.0):
        self._budget = budget_bytes
        self.bpe = bytes_per_element
        self.step_time = step_time
        self.left: Dict[int, int] = {}
        self.poisoned: Dict[int, bool] = {}
        self.next_slot = 0
        self.admitted: List[int] = []
        self.max_used = 0
        self.used = 0
        self.sizes: Dict[int, int] = {}
        self.discarded: List[int] = []
        self.prepared = 0              # footprints of prepared requests not yet admitted or discarded
        self.max_prepared = 0
        self._lock = threading.Lock()

    def footprint(self, req):
        return req.elements * self.bpe

    def budget(self):
        return self._budget

    def prepare(self, req):
        if req.spec.steps <= 0:
            raise ValueError("no steps requested")
        with self._lock:
            self.prepared += self.footprint(req)
            self.max_prepared = max(self.max_prepared, self.prepared)
        return req

    def admit(self, req):
        fp = self.footprint(req)
        assert self.used + fp <= self._budget, "admitted beyond the budget"
        with self._lock:
            self.prepared -= fp
        s = self.next_slot
        self.next_slot += 1
        self.left[s] = req.spec.steps
        self.poisoned[s] = req.poisoned
        self.sizes[s] = fp
        self.used += fp
        self.max_used = max(self.max_used, self.used)
        self.admitted.append(req.rid)
        return s

    def tick(self, nsteps):
        if self.step_time:
            time.sleep(self.step_time * nsteps)
        for s in self.left:
            self.left[s] = max(0, self.left[s] - nsteps)

    def poll(self):
        return [(s, self.poisoned[s]) for s in sorted(self.left) if self.left[s] == 0 or self.poisoned[s]]

    def retire(self, slot, failed):
        self.left.pop(slot)
        self.poisoned.pop(slot)
        self.used -= self.sizes.pop(slot)
        return None, 1.0

    def discard(self, handle):
        self.discarded.append(handle.rid)
        with self._lock:
            self.prepared -= self.footprint(handle)
