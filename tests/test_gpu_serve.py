"""Served mixed stream on the GPU: every frame served in the mix (graphs,
several streams, memory admission) is bitwise identical to the same frame
computed alone by the plain per-frame path."""

import numpy as np
import pytest

import phantom
from phantom.configs import served_pool
from wfhelp import scan_from_workload

pytestmark = pytest.mark.gpu


def test_mixed_stream_matches_alone(wf_gpu):
    import torch

    from paper_1811_01566_amd.serve import (GpuBackend, Request, Server, latency_stats,
                                            poisson_trace, run_plain)

    pool = [w for w in served_pool(8, seed=11)]
    rfs = [torch.from_numpy(phantom.synth_rf(w)[0]).cuda() for w in pool]
    scans = [scan_from_workload(w) for w in pool]
    arrivals, cls = poisson_trace(pool, rate_hz=4000.0, n=48, seed=3)
    reqs = [Request(i, scans[k], rfs[k], float(t), pool[k].dr_db)
            for i, (t, k) in enumerate(zip(arrivals, cls))]
    # a budget that holds only a few executors, to exercise admission and eviction
    budget = 3 * max(rf.numel() * 2 for rf in rfs) + (64 << 20)
    srv = Server(GpuBackend("cuda:0", use_graphs=True), hbm_budget=budget, n_streams=4)
    served = srv.run_trace(reqs)
    torch.cuda.synchronize()
    alone = run_plain(reqs)
    for a, b in zip(served, alone):
        assert a.rid == b.rid
        assert torch.equal(a.image, b.image), f"request {a.rid} differs"
    st = latency_stats(served)
    print(f"served: {st}, executors built {srv.executors_built}, evictions {srv.evictions}, "
          f"waits for memory {srv.waits_for_memory}, max in flight {srv.max_inflight}")
    assert srv.max_inflight > 1
    assert srv.bytes_in_use <= budget
