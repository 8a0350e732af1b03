"""Serving loop bookkeeping on the CPU with a simulated device: admission by
memory, stream slots, eviction, out-of-order admission of other classes,
and latency accounting."""

from dataclasses import dataclass

import pytest

import paper_1811_01566_amd as wf
from paper_1811_01566_amd.serve import Request, Server, frame_bytes, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


@dataclass
class FakeExecutor:
    nbytes: int
    busy: bool = False
    last_used: float = 0.0


class FakeBackend:
    """Each stream runs its requests back to back; a request takes
    `cost(req)` seconds of device time."""

    def __init__(self, clock, cost):
        self.clock = clock
        self.cost = cost
        self.free_at = {}
        self.built = []

    def new_stream(self):
        s = len(self.free_at)
        self.free_at[s] = 0.0
        return s

    def new_executor(self, req):
        ex = FakeExecutor(frame_bytes(req))
        self.built.append(req.rid)
        return ex

    def launch(self, ex, req, stream):
        start = max(self.clock(), self.free_at[stream])
        end = start + self.cost(req)
        self.free_at[stream] = end
        return end, ("image", req.rid)

    def done(self, event):
        return self.clock() >= event


class Shape:
    def __init__(self, n_s):
        self.shape = (4, 8, n_s)


def _scan(n_tx=4, n_ch=8, nz=64, nx=32):
    return wf.Scan(mode="pwi", n_elem=8, pitch=3e-4, c=1540.0, fs=50e6, n_tx=n_tx, n_ch=n_ch,
                   grid=wf.Grid(nz, nx, 5e-3, 1e-4, -1e-3, 1e-4), angles_rad=(0.0,) * n_tx)


def _run(server, reqs, clock, step=1e-4):
    def idle():
        clock.t += step
    return server.run_trace(reqs, clock=clock, idle=idle)


def test_overlap_and_latency_accounting():
    clock = FakeClock()
    be = FakeBackend(clock, cost=lambda r: 1e-3)
    srv = Server(be, hbm_budget=1 << 30, n_streams=4)
    reqs = [Request(i, _scan(), Shape(256), arrival=0.0) for i in range(8)]
    res = _run(srv, reqs, clock)
    assert [r.rid for r in res] == list(range(8))
    assert srv.max_inflight == 4
    # 8 requests of 1 ms on 4 streams: two waves
    lat = sorted(r.latency for r in res)
    assert lat[3] == pytest.approx(1e-3, abs=2e-4)
    assert lat[7] == pytest.approx(2e-3, abs=3e-4)
    st = latency_stats(res)
    assert st["requests"] == 8 and st["p99_ms"] >= st["p50_ms"]


def test_memory_budget_limits_executors_and_evicts_idle():
    clock = FakeClock()
    be = FakeBackend(clock, cost=lambda r: 1e-3)
    a, b = _scan(n_tx=4), _scan(n_tx=2)
    need_a = frame_bytes(Request(0, a, Shape(256), 0.0))
    need_b = frame_bytes(Request(0, b, Shape(256), 0.0))
    # room for two executors of class a, or one of each
    srv = Server(be, hbm_budget=2 * need_a, n_streams=4)
    reqs = [Request(i, a, Shape(256), arrival=0.0) for i in range(3)]
    reqs += [Request(3, b, Shape(256), arrival=0.5e-3)]
    res = _run(srv, reqs, clock)
    assert len(res) == 4
    assert srv.bytes_in_use <= 2 * need_a
    assert srv.waits_for_memory > 0  # the third class-a request waited for memory
    assert srv.evictions >= 1        # class b evicted an idle class-a executor
    assert need_b < need_a


def test_other_classes_overtake_a_request_waiting_for_memory():
    clock = FakeClock()
    be = FakeBackend(clock, cost=lambda r: 2e-3 if r.scan.n_tx == 4 else 0.2e-3)
    big, small = _scan(n_tx=4), _scan(n_tx=1)
    need_big = frame_bytes(Request(0, big, Shape(256), 0.0))
    need_small = frame_bytes(Request(0, small, Shape(256), 0.0))
    srv = Server(be, hbm_budget=need_big + need_small, n_streams=4)
    reqs = [Request(0, big, Shape(256), 0.0), Request(1, big, Shape(256), 0.1e-3),
            Request(2, small, Shape(256), 0.2e-3)]
    res = {r.rid: r for r in _run(srv, reqs, clock)}
    # request 1 cannot get memory until request 0 finishes; request 2 can
    assert res[2].done < res[1].start


def test_oversized_request_is_rejected():
    clock = FakeClock()
    srv = Server(FakeBackend(clock, cost=lambda r: 1e-3), hbm_budget=1000, n_streams=2)
    with pytest.raises(ValueError, match="budget"):
        _run(srv, [Request(0, _scan(), Shape(256), 0.0)], clock)



def test_prewarm_builds_per_class_within_budget():
    clock = FakeClock()
    be = FakeBackend(clock, cost=lambda r: 1e-3)
    srv = Server(be, hbm_budget=1 << 30, n_streams=3)
    # three shape classes (transmit counts 2, 4, 6)
    reqs = [Request(i, _scan(n_tx=2 + 2 * k), Shape(256), arrival=0.0)
            for i, k in enumerate([0, 1, 0, 2, 1])]
    srv.prewarm(reqs)
    assert srv.executors_built == 9  # 3 classes x 3 stream slots
    _run(srv, reqs, clock)
    assert srv.executors_built == 9  # serving built nothing more
    small = Server(FakeBackend(clock, cost=lambda r: 1e-3),
                   hbm_budget=2 * frame_bytes(reqs[0]) + 1, n_streams=3)
    small.prewarm(reqs)
    assert small.executors_built == 2 and small.bytes_in_use <= small.budget
