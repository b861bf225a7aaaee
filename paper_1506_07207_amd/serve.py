"""Continuous-batching request loop for simplex-in-cell simulations.

Requests (independent 1D1V simulations) arrive over time.  The server admits
each one into a resident batch as soon as a slot and its share of the tracer
budget are free, advances every resident simulation together in chunks of
steps, and retires a simulation the moment its own step count is reached,
which frees room for the next arrivals.  A request that arrives while others
are running therefore joins their launches instead of waiting for them.

Batches are split into size classes by cell count: the tracer kernel keeps one
copy of a simulation's mesh in LDS per workgroup, sized for the largest mesh
of its batch, so rare large meshes get a batch of their own and do not lower
the occupancy of the common small ones.

The scheduling logic talks to an executor (``GpuExecutor`` drives libsic;
tests use a fake one on a simulated clock).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, Iterable, List, Optional

import numpy as np

from . import inputs


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    tracers: int
    steps: int
    admitted: float = math.nan
    completed: float = math.nan
    final_W_E: float = math.nan
    flags: int = 0
    size_class: int = -1
    W_E_history: Optional[np.ndarray] = None  # kept when the executor keeps histories

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@dataclasses.dataclass
class Report:
    records: List[Record]
    wall: float
    warmup_fraction: float

    def completed(self) -> List[Record]:
        return [r for r in self.records if not math.isnan(r.completed)]

    def measured(self) -> List[Record]:
        done = sorted(self.completed(), key=lambda r: r.rid)
        skip = int(len(self.records) * self.warmup_fraction)
        return [r for r in done if r.rid >= skip]

    def latency_quantiles(self, qs=(0.5, 0.99)) -> Dict[float, float]:
        lat = np.array([r.latency for r in self.measured()])
        if len(lat) == 0:
            return {q: math.nan for q in qs}
        return {q: float(np.quantile(lat, q)) for q in qs}

    def tracer_updates_per_s(self) -> float:
        done = self.completed()
        if not done:
            return 0.0
        t0 = min(r.arrival for r in self.records)
        t1 = max(r.completed for r in done)
        return sum(r.tracers * r.steps for r in done) / max(t1 - t0, 1e-12)

    def summary(self) -> dict:
        q = self.latency_quantiles()
        return dict(requests=len(self.records), completed=len(self.completed()),
                    measured=len(self.measured()), p50_s=q[0.5], p99_s=q[0.99],
                    tracer_updates_per_s=self.tracer_updates_per_s(), wall_s=self.wall)


class Executor:
    """Interface the request loop drives."""

    def admit(self, req) -> Optional[object]:  # handle, or None when full
        raise NotImplementedError

    def active(self) -> int:
        raise NotImplementedError

    def step(self, n: int) -> None:
        raise NotImplementedError

    def poll(self) -> List[object]:
        raise NotImplementedError

    def finish(self, handle) -> dict:  # final diagnostics; frees the slot
        raise NotImplementedError


class Server:
    """FIFO admission with bounded bypass: when the oldest waiting request
    does not fit, up to ``bypass`` younger ones may be admitted past it, but
    no request is passed over more than ``max_passed`` times (no starvation).
    """

    def __init__(self, executor: Executor, chunk_steps: int = 32, bypass: int = 8, max_passed: int = 64,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.chunk = int(chunk_steps)
        self.bypass = int(bypass)
        self.max_passed = int(max_passed)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests: Iterable, warmup_fraction: float = 0.1, prepare: Optional[Callable] = None,
            progress: Optional[Callable[[int, int], None]] = None) -> Report:
        """Serves the stream in real time; progress(done, total), if given,
        is called each time another tenth of the requests has completed."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        done, step_report = 0, max(1, len(reqs) // 10)
        records = {r.rid: Record(r.rid, r.arrival, r.spec.tracers, r.spec.n_steps) for r in reqs}
        waiting = collections.deque()
        passed: Dict[int, int] = collections.defaultdict(int)
        handles: Dict[object, int] = {}
        nxt = 0
        t0 = self.clock()
        while nxt < len(reqs) or waiting or handles:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            # admission
            tried = 0
            i = 0
            while i < len(waiting) and tried <= self.bypass:
                req = waiting[i]
                if i > 0 and passed[waiting[0].rid] >= self.max_passed:
                    break
                h = self.ex.admit(req)
                tried += 1
                if h is None:
                    i += 1
                    continue
                handles[h] = req.rid
                records[req.rid].admitted = self.clock() - t0
                records[req.rid].size_class = getattr(h, "size_class", -1)
                del waiting[i]
                if i > 0:
                    passed[waiting[0].rid] += 1
            if handles:
                self.ex.step(self.chunk)
                if prepare is not None:
                    prepare(waiting, reqs[nxt:nxt + 64])
                for h in self.ex.poll():
                    rid = handles.pop(h)
                    res = self.ex.finish(h)
                    rec = records[rid]
                    rec.completed = self.clock() - t0
                    rec.final_W_E = float(res.get("W_E", math.nan))
                    rec.flags = int(res.get("flags", 0))
                    rec.W_E_history = res.get("W_E_history")
                    done += 1
                    if progress is not None and done % step_report == 0:
                        progress(done, len(reqs))
            elif nxt < len(reqs):
                wait = reqs[nxt].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
            elif waiting:
                raise RuntimeError(f"request {waiting[0].rid} can never be admitted (larger than the executor)")
        return Report([records[r.rid] for r in reqs], self.clock() - t0, warmup_fraction)


# --------------------------------------------------------------------------- GPU executor

@dataclasses.dataclass(frozen=True)
class SizeClass:
    max_cells: int
    budget_tracers: int
    max_slots: int


DEFAULT_CLASSES = (SizeClass(1024, 1_900_000_000, 8192), SizeClass(4096, 100_000_000, 16))


class _Handle:
    __slots__ = ("size_class", "slot")

    def __init__(self, size_class, slot):
        self.size_class = size_class
        self.slot = slot

    def __hash__(self):
        return hash((self.size_class, self.slot))

    def __eq__(self, o):
        return isinstance(o, _Handle) and (o.size_class, o.slot) == (self.size_class, self.slot)


class GpuExecutor(Executor):
    """Resident batches of libsic, one per size class, on the current stream."""

    def __init__(self, classes=DEFAULT_CLASSES, precision: int = 0, history_rows: int = 4096, autotune=False,
                 keep_history: bool = False):
        import torch

        from . import binding as B

        self.B = B
        self.torch = torch
        self.classes = list(classes)
        self.precision = precision
        self.keep_history = keep_history
        # one stream per size class (default priority): the classes' steps
        # overlap on the device, so the large-mesh class, whose LDS mesh
        # leaves room for few workgroups per CU, shares the GPU with the rest
        self.streams = [torch.cuda.Stream() for _ in self.classes]
        self.batches = [B.sic_batch_create(c.budget_tracers, c.max_slots, c.max_cells, precision=precision,
                                           history_rows=history_rows, stream=st)
                        for c, st in zip(self.classes, self.streams)]
        self.live = [set() for _ in self.classes]
        self.cache: Dict[int, tuple] = {}
        # request arrays are built on a stream of their own (default
        # priority), so building them never waits for the batch's steps
        self.side = torch.cuda.Stream()

    def close(self):
        for b in self.batches:
            self.B.sic_batch_destroy(b)
        self.batches = []

    def _class_of(self, spec) -> int:
        for i, c in enumerate(self.classes):
            if spec.n_cells <= c.max_cells and spec.tracers <= c.budget_tracers:
                return i
        raise ValueError("request larger than every size class")

    def prepare(self, req):
        """Host and device arrays of a request (done ahead of admission, on
        the side stream; the event marks them ready)."""
        if req.rid in self.cache:
            return self.cache[req.rid]
        p = req.spec.build()
        torch = self.torch
        with torch.cuda.stream(self.side):
            line = torch.from_numpy(p.line).to("cuda", non_blocking=True)
            sv = torch.from_numpy(p.sheet_v).to("cuda", non_blocking=True)
            x0 = line.repeat(p.n_sheets)
            v0 = sv.repeat_interleave(int(p.n_tracers[0]))
            ready = torch.cuda.Event()
            ready.record(self.side)
        self.cache[req.rid] = (p, x0, v0, ready)
        return self.cache[req.rid]

    def admit(self, req):
        ci = self._class_of(req.spec)
        p, x0, v0, ready = self.prepare(req)
        ready.synchronize()
        slot = self.B.sic_batch_admit(self.batches[ci], p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, x0, v0,
                                      p.n_steps, precision=self.precision, raise_busy=False)
        if slot is None:
            return None
        self.cache.pop(req.rid, None)
        self.live[ci].add(slot)
        return _Handle(ci, slot)

    def active(self) -> int:
        return sum(len(s) for s in self.live)

    def step(self, n: int) -> None:
        for ci, b in enumerate(self.batches):
            if self.live[ci]:
                self.B.sic_batch_step(b, n)

    def poll(self):
        out = []
        for ci, b in enumerate(self.batches):
            if self.live[ci]:
                out += [_Handle(ci, s) for s in self.B.sic_batch_poll(b)]
        return out

    def finish(self, h) -> dict:
        b = self.batches[h.size_class]
        r = self.B.sic_batch_result(b, h.slot, history=self.keep_history)
        self.B.sic_batch_release(b, h.slot)
        self.live[h.size_class].discard(h.slot)
        out = dict(r["last"])
        if self.keep_history:
            out["W_E_history"] = np.array(r["history"]["W_E"])
        return out


def serve_prepare(executor: GpuExecutor):
    """Hook that builds the arrays of waiting and soon-to-arrive requests
    while the GPU runs a chunk of steps."""

    def prepare(waiting, upcoming):
        for r in list(waiting)[:16]:
            executor.prepare(r)
        for r in upcoming[:8]:
            executor.prepare(r)

    return prepare


# --------------------------------------------------------------------------- plain baseline

def serve_plain(requests: Iterable, precision: int = 0, clock=time.perf_counter, sleep=time.sleep) -> Report:
    """The same stream served one request at a time, each as its own
    simulation with its own launches (no batching)."""
    import torch

    from . import binding as B

    reqs = sorted(requests, key=lambda r: r.arrival)
    records = [Record(r.rid, r.arrival, r.spec.tracers, r.spec.n_steps) for r in reqs]
    t0 = clock()
    for rec, r in zip(records, reqs):
        now = clock() - t0
        if r.arrival > now:
            sleep(r.arrival - now)
        p = r.spec.build()
        x0 = torch.from_numpy(p.line).cuda().repeat(p.n_sheets)
        v0 = torch.from_numpy(p.sheet_v).cuda().repeat_interleave(int(p.n_tracers[0]))
        rec.admitted = clock() - t0
        with B.Simulation(p, precision=precision, history_rows=64, x0=x0, v0=v0) as s:
            s.step(p.n_steps)
            last = s.diagnostics(history=False)["last"]
        rec.completed = clock() - t0
        rec.final_W_E = last["W_E"]
        rec.flags = last["flags"]
    return Report(records, clock() - t0, 0.1)


def poisson_stream(n_requests: int, rate: float, seed: int = 20251204, p_large: float = 0.005):
    return list(inputs.request_stream(n_requests, rate, seed=seed, p_large=p_large))
