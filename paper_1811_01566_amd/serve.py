"""Continuous-batching service for a mixed stream of B-mode frame requests.

Requests of different geometries (array size, transmit count, record length,
pixel grid, STAI or PWI) arrive over time.  The service keeps, per shape
class, resident executors: a plan of the geometry (constant tables, work
list and, where they are small against the memory budget, the delay tables,
in device memory the executor owns), device buffers for one frame (RF
in, beamformed RF, B-mode out, column maxima, the DAS work-split workspace)
and a HIP graph of the whole path (DAS -> envelope -> log compression),
captured on the executor's first call and replayed per request.  Up to ``n_streams`` requests are in
flight at once, each on its own stream, so a request that arrives while
others run is admitted as soon as a stream slot and memory are free, and its
kernels overlap with theirs on the device.

Memory admission: every executor is charged its buffer bytes against
``hbm_budget``.  A class without an idle executor gets a new one if the
budget allows, after evicting idle executors of other classes (least
recently used first); otherwise the request waits and later arrivals of
other classes may go first.

Results are deterministic: the forward path has no atomics and a fixed
accumulation order, so a frame served in the mix is bitwise identical to the
same frame computed alone.

:func:`run_plain` is the plain per-frame path: one request at a time in
arrival order on one stream, no graphs.  Both report latency from arrival to
completion of each request.

The device work goes through a small backend interface (:class:`GpuBackend`)
so that admission, scheduling and bookkeeping can be exercised on the CPU
with a simulated device.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

from . import Plan, Scan, bmode, das, das_workspace_bytes, plan_bytes


@dataclass
class Request:
    rid: int
    scan: Scan
    rf: "object"  # int16 [T][C][S] (device tensor for the GPU backend)
    arrival: float  # seconds on the trace clock
    dr_db: float = 60.0

    @property
    def n_s(self) -> int:
        return int(self.rf.shape[-1])


@dataclass
class Result:
    rid: int
    image: "object"  # float32 [nz][nx] B-mode (device tensor)
    arrival: float
    start: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def class_key(req: Request) -> tuple:
    s, g = req.scan, req.scan.grid
    return (s.mode, s.n_elem, s.pitch, s.c, s.fs, s.n_tx, s.n_ch, req.n_s, g.nz, g.nx, g.z0,
            g.dz, g.x0, g.dx, s.t0, s.f_number, tuple(s.tx_elem or ()),
            tuple(s.angles_rad or ()), s.tref, tuple(s.rx_elem or ()), req.dr_db)


def frame_bytes(req: Request) -> int:
    """Device bytes of one executor: int16 RF in, fp32 beamformed and B-mode
    frames, fp32 column maxima."""
    g = req.scan.grid
    return req.scan.n_tx * req.scan.n_ch * req.n_s * 2 + g.nz * g.nx * 8 + g.nx * 4


class Executor:
    """Plan, buffers and (with graphs) a captured replay for one frame of
    one shape class.  The plan's device tables live as long as the executor
    and its graph."""

    def __init__(self, req: Request, device, use_graph: bool, delay_tables: bool = False):
        import torch

        g = req.scan.grid
        self.scan = req.scan
        self.dr_db = req.dr_db
        self.plan = Plan(req.scan, req.n_s, device=device, delay_tables=delay_tables)
        self.rf = torch.zeros((1, req.scan.n_tx, req.scan.n_ch, req.n_s), dtype=torch.int16,
                              device=device)
        self.y = torch.empty((1, g.nz, g.nx), dtype=torch.float32, device=device)
        self.out = torch.empty_like(self.y)
        self.col_max = torch.empty((1, g.nx), dtype=torch.float32, device=device)
        wsb = self.plan.workspace_bytes(1)[0]
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=device) if wsb else None
        self.nbytes = frame_bytes(req) + wsb + self.plan.mem.numel()
        self.graph = None
        self.busy = False
        self.last_used = 0.0
        # the plan's tables were written on the current stream; with the
        # plan the path only enqueues kernels, so its first call is captured
        torch.cuda.synchronize(device)
        if use_graph:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._launch()
            torch.cuda.synchronize(device)

    def _launch(self):
        das(self.scan, self.rf, out=self.y, workspace=self.ws, plan=self.plan)
        bmode(self.y, self.dr_db, out=self.out, col_max=self.col_max)

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self._launch()


class GpuBackend:
    """Streams, events and executors on one GPU.  An executor's plan holds
    the delay tables (see :class:`Plan`) when they take at most
    ``table_limit`` bytes; the :class:`Server` sets it to a sixteenth of its
    HBM budget."""

    def __init__(self, device="cuda:0", use_graphs: bool = True):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.use_graphs = use_graphs
        self.table_limit = 0

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def _delay_tables(self, req: Request) -> bool:
        extra = plan_bytes(req.scan, req.n_s, True) - plan_bytes(req.scan, req.n_s, False)
        return extra <= self.table_limit

    def new_executor(self, req: Request) -> Executor:
        return Executor(req, self.device, self.use_graphs, self._delay_tables(req))

    def executor_bytes(self, req: Request) -> int:
        return (frame_bytes(req) + das_workspace_bytes(req.scan, req.n_s, 1) +
                plan_bytes(req.scan, req.n_s, self._delay_tables(req)))

    def launch(self, ex: Executor, req: Request, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            ex.rf[0].copy_(req.rf, non_blocking=True)
            ex.run()
            image = ex.out[0].clone()
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, image

    def done(self, event) -> bool:
        return bool(event.query())


@dataclass
class _InFlight:
    req: Request
    ex: object
    slot: int
    event: object
    image: object
    start: float


class Server:
    """Admission by memory, executors per shape class, stream slots and
    completion tracking."""

    def __init__(self, backend=None, hbm_budget: int = 8 << 30, n_streams: int = 4):
        self.backend = backend if backend is not None else GpuBackend()
        self.budget = int(hbm_budget)
        if hasattr(self.backend, "table_limit"):
            self.backend.table_limit = self.budget // 16
        self.streams = [self.backend.new_stream() for _ in range(n_streams)]
        self.free_slots = list(range(n_streams))
        self.executors: Dict[tuple, List[object]] = collections.defaultdict(list)
        self.bytes_in_use = 0
        self.inflight: List[_InFlight] = []
        self.queue: collections.deque = collections.deque()
        self.results: List[Result] = []
        self.waits_for_memory = 0
        self.executors_built = 0
        self.evictions = 0
        self.max_inflight = 0

    # -- memory ------------------------------------------------------------
    def _bytes_of(self, req: Request) -> int:
        size = getattr(self.backend, "executor_bytes", None)
        return size(req) if size is not None else frame_bytes(req)

    def _evict_for(self, need: int) -> bool:
        idle = sorted(((ex.last_used, key, ex) for key, lst in self.executors.items()
                       for ex in lst if not ex.busy), key=lambda t: t[0])
        for _, key, ex in idle:
            if self.bytes_in_use + need <= self.budget:
                break
            self.executors[key].remove(ex)
            self.bytes_in_use -= ex.nbytes
            self.evictions += 1
        return self.bytes_in_use + need <= self.budget

    def _executor(self, req: Request):
        key = class_key(req)
        for ex in self.executors[key]:
            if not ex.busy:
                return ex
        need = self._bytes_of(req)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} bytes, above the HBM budget")
        if not self._evict_for(need):
            self.waits_for_memory += 1
            return None
        ex = self.backend.new_executor(req)
        self.executors_built += 1
        self.executors[key].append(ex)
        self.bytes_in_use += ex.nbytes
        return ex

    def prewarm(self, requests: Sequence[Request], per_class: Optional[int] = None) -> None:
        """Build up to `per_class` executors (default: one per stream slot)
        for every shape class in `requests`, within the HBM budget, so that
        no executor - with its synchronising warm-up and graph capture - is
        built while a trace is served."""
        per_class = len(self.streams) if per_class is None else per_class
        seen = {}
        for r in requests:
            seen.setdefault(class_key(r), r)
        for key, r in seen.items():
            while len(self.executors[key]) < per_class:
                need = self._bytes_of(r)
                if self.bytes_in_use + need > self.budget:
                    return
                ex = self.backend.new_executor(r)
                self.executors_built += 1
                self.executors[key].append(ex)
                self.bytes_in_use += ex.nbytes

    # -- scheduling ----------------------------------------------------------
    def submit(self, req: Request) -> None:
        self.queue.append(req)

    def admit(self, clock: Callable[[], float]) -> None:
        waiting = collections.deque()
        while self.queue:
            req = self.queue.popleft()
            ex = self._executor(req) if self.free_slots else None
            if ex is None:
                waiting.append(req)
                continue
            slot = self.free_slots.pop()
            ex.busy = True
            start = clock()
            ex.last_used = start
            ev, image = self.backend.launch(ex, req, self.streams[slot])
            self.inflight.append(_InFlight(req, ex, slot, ev, image, start))
            self.max_inflight = max(self.max_inflight, len(self.inflight))
        self.queue = waiting

    def complete(self, clock: Callable[[], float]) -> int:
        keep, n = [], 0
        for f in self.inflight:
            if self.backend.done(f.event):
                f.ex.busy = False
                self.free_slots.append(f.slot)
                self.results.append(Result(f.req.rid, f.image, f.req.arrival, f.start, clock()))
                n += 1
            else:
                keep.append(f)
        self.inflight = keep
        return n

    def run_trace(self, requests: Sequence[Request], clock: Optional[Callable[[], float]] = None,
                  idle: Optional[Callable[[], None]] = None) -> List[Result]:
        """Replay requests at their arrival times (seconds from the start)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        if clock is None:
            t0 = time.perf_counter()
            clock = lambda: time.perf_counter() - t0  # noqa: E731
        i, n = 0, len(reqs)
        target = len(self.results) + n
        while len(self.results) < target:
            now = clock()
            while i < n and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self.admit(clock)
            if self.complete(clock) == 0 and idle is not None:
                idle()
        return sorted(self.results[-n:], key=lambda r: r.rid)


def run_plain(requests: Sequence[Request], device="cuda:0") -> List[Result]:
    """One request at a time, in arrival order, on one stream, no graphs."""
    import torch

    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    out = []
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            pass
        start = time.perf_counter() - t0
        y = das(r.scan, r.rf)
        img = bmode(y, r.dr_db)
        torch.cuda.synchronize(device)
        out.append(Result(r.rid, img, r.arrival, start, time.perf_counter() - t0))
    return sorted(out, key=lambda r: r.rid)


def latency_stats(results: Sequence[Result]) -> dict:
    import numpy as np

    lat = np.array([r.latency for r in results]) * 1e3
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "throughput_rps": len(results) / span if span > 0 else float("nan")}


def poisson_trace(classes: Sequence[tuple], rate_hz: float, n: int, seed: int = 0):
    """Arrival times and class indices of a Poisson stream over `classes`
    (chosen uniformly)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    return np.cumsum(gaps) - gaps[0], rng.integers(0, len(classes), n)
