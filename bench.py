"""Benchmark of the DAS -> envelope -> log-compression B-mode path on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pwi]
                    [--no-cpu-baseline] [--latency-frames N] [--h2d-frames N]

A step is one frame through the whole hot path - DAS (PWI or STAI), the FFT
analytic-signal envelope with per-column maxima, and the dB log compression
with clipping - on int16 RF already resident in HBM.  Default workload: PWI,
64 plane waves over +-16 deg x 128 channels x 2048 samples, 1024 x 512 grid
over 5-30 mm, synthetic cyst phantom (seeded).

Prints ONE JSON line (rank 0) with the B-mode frame rate, DAS throughput in
nominal contributions per second (pixel x transmit x channel), frame latency
percentiles, a roofline object for the dominant kernel (DAS, bound by the
vector ALU) and the FP64 CPU oracle timed on a bounded sample of the same
frame.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz retire 39.3e12 vector
# lane-instructions per second without packed-FP32 dual issue; the published
# 157.3 TFLOP/s FP32 vector peak is that rate x 2 (FMA) x 2 (packed).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12  # bytes/s
# non-packed FP32 fused multiply-add rate: 2 flops per lane-instruction
PEAK_FMA = 2 * PEAK_LANE_OPS
# algorithmic lane-ops of one active contribution: transmit + receive delay
# add, index / fraction split, r[n+1] - r[n], interpolating FMA, accumulate
OPS_PER_CONTRIB = 5
# shape classes of the short served-stream summary on the single-workload line
SUMMARY_CLASSES = 8

PAPER_CONTEXT = {
    "source": "WaveFlow (arXiv 1811.01566) Table I, NVIDIA Titan X, TF 1.6, float64 input",
    "stai_fps": 55, "pwi_fps": 17,
    "stai_shape": "(128, 64, 2048) -> (2048, 128)", "pwi_shape": "(11, 192, 2048) -> (512, 128)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="pwi", choices=["pwi", "stai_full", "stai_small",
                                                          "pwi_batch8", "paper_stai",
                                                          "paper_pwi"])
    ap.add_argument("--rf-dtype", default="int16", choices=["int16", "float16", "float32"],
                    help="RF storage: int16 ADC counts, FP16 (counts x 2^-13) or FP32")
    ap.add_argument("--latency-frames", type=int, default=1000)
    ap.add_argument("--h2d-frames", type=int, default=20,
                    help="frames of the PCIe-inclusive section (0 leaves it out, e.g. under a "
                         "kernel trace, whose per-kernel averages it would mix with launches "
                         "that overlap host copies)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-columns", type=int, default=64,
                    help="image columns of the frame the one-core CPU oracle computes")
    ap.add_argument("--cpu-pool-columns", type=int, default=512,
                    help="image columns of the frame the all-cores CPU oracle computes")
    ap.add_argument("--serve", action="store_true",
                    help="served mixed stream (continuous batching) vs the plain per-frame "
                         "path instead of the single-workload benchmark")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-classes", type=int, default=16)
    ap.add_argument("--serve-load", type=float, default=0.75,
                    help="arrival rate as a fraction of the plain path's capacity")
    ap.add_argument("--serve-summary", type=int, default=300, metavar="REQUESTS",
                    help="requests of the short served-stream summary added to the "
                         "single-workload line (8 shape classes; 0 leaves it out)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, 5 times (reference "
                         "for the HBM byte counters), and exit")
    return ap.parse_args()


def active_contributions(w):
    """Pixel x transmit x channel triples whose echo sample lies inside the
    record and whose channel is inside the receive aperture (float64)."""
    import numpy as np

    import oracle

    g = w.grid()
    # every 8th row and column is an unbiased sample of the fraction
    iz = np.arange(0, w.nz, 8)
    ix = np.arange(0, w.nx, 8)
    IZ, IX = np.meshgrid(iz, ix, indexing="ij")
    ttx, trx = oracle.workload_tof(w, IZ, IX)
    x = g["x0"] + IX * g["dx"]
    z = g["z0"] + IZ * g["dz"]
    ex = oracle.element_positions(w.n_elem, w.pitch)[w.rx_elements()]
    act = 0
    for t in range(w.n_tx):
        u = (ttx[t][None] + trx - w.t0) * w.fs
        n = np.floor(u)
        ok = (n >= 0) & (n <= w.n_s - 2)
        if w.f_number > 0:
            ok &= 2 * w.f_number * np.abs(x[None] - ex[:, None, None]) <= z[None]
        act += int(ok.sum())
    frac = act / (w.n_tx * w.n_ch * IZ.size)
    return frac


KERNEL_SOURCES = ("das.hip", "das_common.h", "ff.h", "wf_internal.h")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1811_01566_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str):
    """HBM bytes per DAS launch from the committed rocprofv3 counter summary
    of this workload, scaled by the copy-kernel calibration; None when the
    summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"das_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha1") != kernel_source_hash():
        return None
    try:
        fetch = float(kv["fetch_kib_per_launch"]) * float(kv["copy_fetch_factor"])
        write = float(kv["write_kib_per_launch"]) * float(kv["copy_write_factor"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


def scan_of(wf, w):
    """Binding geometry of a synthetic workload."""
    g = w.grid()
    kw = dict(mode=w.mode, n_elem=w.n_elem, pitch=w.pitch, c=w.c, fs=w.fs, n_tx=w.n_tx,
              n_ch=w.n_ch, grid=wf.Grid(g["nz"], g["nx"], g["z0"], g["dz"], g["x0"], g["dx"]),
              t0=w.t0, f_number=w.f_number,
              rx_elem=tuple(w.rx_elem) if w.rx_elem is not None else None)
    if w.mode == "stai":
        kw["tx_elem"] = tuple(w.tx_elements())
    else:
        kw["angles_rad"] = tuple(w.angles_rad())
        kw["tref"] = w.tref
    return wf.Scan(**kw)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU_RF = None  # frame-0 RF (float64) the forked oracle workers read


def _oracle_columns(args):
    """The FP64 oracle (DAS, envelope, log compression) on whole columns."""
    import numpy as np

    import oracle

    w, cols = args
    cols = np.asarray(cols)
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(cols, (w.nz, 1))
    y = oracle.das_workload(_CPU_RF, w, iz, ix)
    oracle.log_compress(oracle.envelope(y), w.dr_db)
    return len(cols)


def cpu_baseline(w, rf, ncols, pool_columns):
    """The FP64 oracle timed on the host: on one core over `ncols` whole
    columns of one frame, and with a process pool over every host core the
    process may use (up to 16) over `pool_columns` columns, each scaled to
    frames/s.  Run before the GPU is initialised (the pool forks)."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    global _CPU_RF
    _CPU_RF = rf[0].astype(np.float64)
    try:
        cols = np.linspace(0, w.nx - 1, ncols).round().astype(int)
        t0 = time.perf_counter()
        _oracle_columns((w, cols))
        dt1 = time.perf_counter() - t0
        s1 = dt1 * w.nx / ncols
        cores = max(1, min(len(os.sched_getaffinity(0)), 16))
        pcols = np.linspace(0, w.nx - 1, pool_columns).round().astype(int)
        blocks = [pcols[i::cores * 4] for i in range(cores * 4)]
        blocks = [b for b in blocks if len(b)]
        with ProcessPoolExecutor(max_workers=cores) as ex:
            list(ex.map(_oracle_columns, [(w, blocks[0][:1])] * cores))  # workers up
            t0 = time.perf_counter()
            done = sum(ex.map(_oracle_columns, [(w, b) for b in blocks]))
            dtn = time.perf_counter() - t0
        sn = dtn * w.nx / done
    finally:
        _CPU_RF = None
    return {
        "value": 1.0 / sn, "unit": "frames/s", "cores": cores, "kind": "oracle",
        "sample": f"{done} of {w.nx} columns x {w.nz} rows of one frame, all {w.n_tx}x{w.n_ch} "
                  f"transmit/channel pairs, float64 NumPy, column blocks over a pool of "
                  f"{cores} processes, {dtn:.1f} s measured, scaled by {w.nx}/{done}",
        "s_per_frame": sn,
        "single_core": {"value": 1.0 / s1, "unit": "frames/s", "cores": 1,
                        "sample": f"{ncols} of {w.nx} columns, {dt1:.1f} s measured, scaled by "
                                  f"{w.nx}/{ncols}", "s_per_frame": s1},
        "host_cpus": len(os.sched_getaffinity(0)),
        "host_cpu_count": os.cpu_count(),
        "host_cpu_model": host_cpu_model(),
    }


def served_stream(wf, phantom, torch, np, n_classes, n_requests, load, n_warm, n_burst,
                  n_check):
    """Served mixed stream: Poisson arrivals over a seeded pool of shape
    classes (speckle + cyst phantoms) at `load` x the plain path's capacity;
    the server (continuous batching, graphs, 4 streams) and the plain
    per-frame path replay the same trace and report per-request latency
    (arrival -> completion).  Returns the summary."""
    from phantom.configs import served_pool

    from paper_1811_01566_amd.serve import (GpuBackend, Request, Server, latency_stats,
                                            poisson_trace, run_plain)

    pool = served_pool(n_classes)
    dev = torch.device("cuda:0")
    rfs = [torch.from_numpy(phantom.synth_rf(w)[0]).to(dev) for w in pool]
    scans = [scan_of(wf, w) for w in pool]
    # plain service time per class (the capacity the arrival rate refers to)
    svc = []
    for sc, rf, w in zip(scans, rfs, pool):
        for _ in range(3):
            wf.bmode(wf.das(sc, rf), w.dr_db)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            wf.bmode(wf.das(sc, rf), w.dr_db)
            torch.cuda.synchronize()
        svc.append((time.perf_counter() - t) / 10)
    capacity = 1.0 / float(np.mean(svc))
    rate = load * capacity
    arrivals, cls = poisson_trace(pool, rate, n_requests, seed=5)
    reqs = [Request(i, scans[k], rfs[k], float(t), pool[k].dr_db)
            for i, (t, k) in enumerate(zip(arrivals, cls))]
    print(f"[bench] serve: {len(pool)} classes, plain capacity {capacity:.0f} frames/s, "
          f"arrival rate {rate:.0f}/s, {len(reqs)} requests", file=sys.stderr, flush=True)
    budget = 16 << 30
    srv = Server(GpuBackend("cuda:0", use_graphs=True), hbm_budget=budget, n_streams=4)
    srv.prewarm(reqs)  # executors (buffers + captured graphs) for every class
    srv.run_trace(reqs[: min(n_warm, len(reqs))])  # warm-up
    srv.results.clear()
    built_before = srv.executors_built
    served = latency_stats(srv.run_trace(reqs))
    built_during = srv.executors_built - built_before
    plain = latency_stats(run_plain(reqs))
    ok = all(torch.equal(a.image, b.image) for a, b in
             zip(srv.run_trace(reqs[:n_check]), run_plain(reqs[:n_check])))
    # saturation: the same requests all arriving at once
    burst = [Request(r.rid, r.scan, r.rf, 0.0, r.dr_db) for r in reqs[: min(n_burst, len(reqs))]]
    served_sat = latency_stats(srv.run_trace(burst))["throughput_rps"]
    plain_sat = latency_stats(run_plain(burst))["throughput_rps"]
    return {
        "classes": [w.name for w in pool], "requests": len(reqs),
        "arrival": f"Poisson, {load:.2f} x plain capacity",
        "streams": 4, "hbm_budget_bytes": budget, "graphs": True,
        "served": served, "plain": plain,
        "plain_capacity_fps": capacity, "arrival_rate_hz": rate,
        "saturation_fps": {"served": round(served_sat, 2), "plain": round(plain_sat, 2),
                           "requests": len(burst)},
        "served_equals_plain_bitwise": bool(ok),
        "executors_built": srv.executors_built,
        "executors_built_during_trace": built_during, "max_in_flight": srv.max_inflight,
    }


def serve_main(args, wf, phantom, torch, np):
    """The served mixed stream as the headline of its own JSON line."""
    s = served_stream(wf, phantom, torch, np, args.serve_classes, args.serve_requests,
                      args.serve_load, 200, 600, 64)
    served = s["served"]
    res = {
        "metric": "B-mode frames/s + DAS Gsamples/s (PWI 128ch×64tx); p99 frame latency",
        "value": round(served["throughput_rps"], 2), "unit": "frames/s",
        "n_gpus": 1, "steps": s["requests"], "warmup": 200,
        "ms_per_step": round(1e3 / served["throughput_rps"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "served_mixed_stream", "classes": s["classes"],
                   "arrival": s["arrival"], "streams": s["streams"],
                   "hbm_budget_bytes": s["hbm_budget_bytes"], "graphs": True},
    }
    res.update({k: v for k, v in s.items()
                if k not in ("classes", "arrival", "streams", "hbm_budget_bytes", "graphs")})
    print(json.dumps(res), flush=True)


def pcie_inclusive(wf, torch, scan, w, rf, y, out, col_max, das_ws, stream, n_h2d):
    """Frames/s with the RF streamed from pinned host memory: frame i's RF is
    copied on a second stream into one of two device buffers while frame i-1
    is processed.  The headline value keeps the RF resident in HBM."""
    if n_h2d <= 0:
        return None
    dev = rf.device
    # allocated pinned and filled by a device-to-host copy: no bulk memcpy on
    # host threads right before the timed loop
    host_rf = torch.empty(rf.shape, dtype=rf.dtype, pin_memory=True)
    host_rf.copy_(rf)
    copy_stream = torch.cuda.Stream(device=dev)
    bufs = [torch.empty_like(rf) for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    freed = [torch.cuda.Event() for _ in range(2)]
    for ev in freed:
        ev.record(stream)
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(copy_stream):
        h0.record(copy_stream)
        bufs[0].copy_(host_rf, non_blocking=True)
        h1.record(copy_stream)
    copy_stream.synchronize()
    h2d_ms = h0.elapsed_time(h1)

    def frames(n):
        enqueue_max = 0.0
        for i in range(n):
            t_i = time.perf_counter()
            b = i % 2
            with torch.cuda.stream(copy_stream):
                copy_stream.wait_event(freed[b])
                bufs[b].copy_(host_rf, non_blocking=True)
                copied[b].record(copy_stream)
            stream.wait_event(copied[b])
            wf.das(scan, bufs[b], out=y, workspace=das_ws)
            freed[b].record(stream)
            wf.bmode(y, w.dr_db, out=out, col_max=col_max)
            enqueue_max = max(enqueue_max, time.perf_counter() - t_i)
        torch.cuda.synchronize()
        return enqueue_max

    # untimed pass first: the runtime sets up the copy stream and grows its
    # per-queue resources the first time the host runs many frames ahead,
    # which blocks the enqueueing thread for several ms
    frames(n_h2d)
    t_h = time.perf_counter()
    enqueue_max = frames(n_h2d)
    fps = w.n_frames * n_h2d / (time.perf_counter() - t_h)
    return {"frames_per_s": round(fps, 2), "h2d_ms_per_step": round(h2d_ms, 4),
            "rf_bytes_per_step": int(rf.numel() * rf.element_size()),
            "frames": n_h2d, "host_enqueue_ms_max": round(enqueue_max * 1e3, 3),
            "note": "RF copied from pinned host memory on a second stream, "
                    "double-buffered against DAS + B-mode; timed after one untimed "
                    "pass of the same loop"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the DAS path needs no collective and the "
              "benchmark measures a single MI355X (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_01566_amd as wf
    import phantom

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 4 * n, "launches": 5}), flush=True)
        return

    if args.serve:
        from phantom.configs import served_pool

        for w0 in served_pool(args.serve_classes):  # before the GPU is initialised
            phantom.synth_rf(w0)
        if not torch.cuda.is_available():
            print("no GPU visible", file=sys.stderr)
            sys.exit(1)
        wf.load()
        serve_main(args, wf, phantom, torch, np)
        return

    w = phantom.get_workload(args.workload)
    # synthesise before the GPU is initialised (the generator forks workers)
    if args.serve_summary:
        from phantom.configs import served_pool

        for w0 in served_pool(SUMMARY_CLASSES):
            phantom.synth_rf(w0)
    print(f"[bench] synthesising {w.name} RF ...", file=sys.stderr, flush=True)
    t_syn = time.perf_counter()
    rf_np = phantom.synth_rf(w)
    print(f"[bench] RF {rf_np.shape} {rf_np.dtype} in {time.perf_counter() - t_syn:.1f} s",
          file=sys.stderr, flush=True)
    # the host baseline forks a worker pool: before the GPU is initialised
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, rf_np, args.cpu_columns, min(args.cpu_pool_columns, w.nx))
        print(f"[bench] CPU oracle: {cpu['s_per_frame']:.2f} s/frame on {cpu['cores']} cores, "
              f"{cpu['single_core']['s_per_frame']:.2f} s/frame on one", file=sys.stderr,
              flush=True)
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    wf.load()
    dev = torch.device("cuda:0")

    scan = scan_of(wf, w)
    rf = torch.from_numpy(rf_np).to(dev)
    if args.rf_dtype == "float16":
        rf = (rf.float() * 2.0 ** -13).half()
    elif args.rf_dtype == "float32":
        rf = rf.float()
    F = w.n_frames
    y = torch.empty((F, w.nz, w.nx), dtype=torch.float32, device=dev)
    out = torch.empty_like(y)
    col_max = torch.empty((F, w.nx), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    wsb = wf.das_workspace_bytes(scan, w.n_s, F)
    das_ws = torch.empty(wsb, dtype=torch.uint8, device=dev) if wsb else None

    def step():
        wf.das(scan, rf, out=y, workspace=das_ws)
        wf.bmode(y, w.dr_db, out=out, col_max=col_max)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps, per-kernel HIP events on the same stream --
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        wf.das(scan, rf, out=y, workspace=das_ws)
        ev[i][1].record(stream)
        wf.bmode(y, w.dr_db, out=out, col_max=col_max)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    das_ms = [a.elapsed_time(b) for a, b, _ in ev]
    post_ms = [b.elapsed_time(c) for _, b, c in ev]
    ms_per_step = wall * 1e3 / args.steps

    # ---- per-kernel split of the post-processing (Table I analogue) -------
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    env_ms, logc_ms = [], []
    for _ in range(10):
        e0.record(stream)
        wf.envelope(y, env=out, col_max=col_max)
        e1.record(stream)
        wf.log_compress(out, col_max, w.dr_db, out=out)
        e2.record(stream)
        torch.cuda.synchronize()
        env_ms.append(e0.elapsed_time(e1))
        logc_ms.append(e1.elapsed_time(e2))

    # ---- FIR pre-filter and qUS moment maps, timed beside the B-mode step -
    from phantom.configs import FIR_TAPS, QUS_WINDOW

    taps = phantom.workload_taps(w, FIR_TAPS)
    rf_f = torch.empty(rf.shape, dtype=torch.float32, device=dev)
    env_buf, _ = wf.envelope(y)
    q = QUS_WINDOW
    fir_ms, mom_ms = [], []
    for i in range(12):
        e0.record(stream)
        wf.fir(rf, taps, out=rf_f)
        e1.record(stream)
        maps = wf.moments(env_buf, q["wz"], q["wx"], q["sz"], q["sx"])
        e2.record(stream)
        torch.cuda.synchronize()
        if i >= 2:
            fir_ms.append(e0.elapsed_time(e1))
            mom_ms.append(e1.elapsed_time(e2))
    fir_s = float(np.mean(fir_ms)) * 1e-3
    n_samp = rf.numel()
    fir_bytes = n_samp * (rf.element_size() + 4)
    fir_flops = 2.0 * FIR_TAPS * n_samp
    prefilter = {
        "fir": {"ms": round(fir_s * 1e3, 4), "taps": FIR_TAPS,
                "hbm_bytes": fir_bytes, "flops": fir_flops,
                "hbm_frac": round(fir_bytes / fir_s / PEAK_HBM, 4),
                "fma_frac": round(fir_flops / fir_s / PEAK_FMA, 4)},
        "moments": {"ms": round(float(np.mean(mom_ms)), 4), "window": q,
                    "maps": list(maps.shape),
                    "hbm_bytes": int(env_buf.numel() * 4 + maps.numel() * 4)},
    }
    del rf_f

    # ---- derivatives: adjoint (d L / d rf) and forward-mode d y / d c -------
    gcot = torch.randn(y.shape, generator=torch.Generator(device=dev).manual_seed(3),
                       device=dev)
    grad_rf = torch.empty(rf.shape, dtype=torch.float32, device=dev)
    adj_ws = torch.empty(wf.adjoint_workspace_bytes(scan, w.n_s), dtype=torch.uint8, device=dev)
    dydc = torch.empty_like(y)
    adj_ms, dydc_ms = [], []
    for i in range(8):
        e0.record(stream)
        wf.das_adjoint(scan, gcot, w.n_s, out=grad_rf, workspace=adj_ws)
        e1.record(stream)
        wf.das_dydc(scan, rf, out=dydc, workspace=das_ws)
        e2.record(stream)
        torch.cuda.synchronize()
        if i >= 2:
            adj_ms.append(e0.elapsed_time(e1))
            dydc_ms.append(e1.elapsed_time(e2))
    derivatives = {
        "adjoint_ms": round(float(np.mean(adj_ms)), 4),
        "adjoint_note": "per-tile LDS windows to a workspace, then a per-row sum in tile order",
        "adjoint_workspace_bytes": int(adj_ws.numel()),
        "dydc_ms": round(float(np.mean(dydc_ms)), 4),
        "adjoint_gcontrib_per_s": round(w.nominal_contributions / (np.mean(adj_ms) * 1e-3)
                                        / 1e9, 1),
    }
    del grad_rf, adj_ws

    # ---- secondary: RF streamed from pinned host memory (PCIe-inclusive) -
    pcie = pcie_inclusive(wf, torch, scan, w, rf, y, out, col_max, das_ws, stream,
                          args.h2d_frames)

    # ---- closed-loop frame latency: enqueue -> completion, one in flight --
    lat = []
    for _ in range(args.latency_frames):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.asarray(lat)

    # ---- short served mixed stream beside the headline (p50 / p99) ----------
    serve_summary = None
    if args.serve_summary:
        serve_summary = served_stream(wf, phantom, torch, np, SUMMARY_CLASSES,
                                      args.serve_summary, 0.75, 50, 200, 16)

    fps = F * args.steps / wall
    das_avg_s = float(np.mean(das_ms)) * 1e-3
    nominal = w.nominal_contributions
    act_frac = active_contributions(w)
    achieved = OPS_PER_CONTRIB * act_frac * nominal / das_avg_s
    res = {
        "metric": "B-mode frames/s + DAS Gsamples/s (PWI 128ch×64tx); p99 frame latency",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "mode": w.mode, "frames_per_step": F, "n_tx": w.n_tx, "n_ch": w.n_ch,
            "n_s": w.n_s, "grid": [w.nz, w.nx], "rf_dtype": args.rf_dtype,
            "depth_mm": [w.z_min * 1e3, w.z_max * 1e3], "f_number": w.f_number,
            "dr_db": w.dr_db, "channel_split_workspace_bytes": wsb,
        },
        "das_gsamples_per_s": round(nominal / das_avg_s / 1e9, 2),
        "das_gsamples_per_s_active": round(act_frac * nominal / das_avg_s / 1e9, 2),
        "active_fraction": round(act_frac, 4),
        "step_ms": {"das": round(float(np.mean(das_ms)), 4),
                    "envelope": round(float(np.mean(env_ms)), 4),
                    "log_compress": round(float(np.mean(logc_ms)), 4),
                    "envelope_plus_log": round(float(np.mean(post_ms)), 4)},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "frames": int(lat.size)},
        "roofline": {
            "bound": "alu",
            "kernel": "das_kernel",
            "achieved": round(achieved / 1e12, 3),
            "peak": round(PEAK_LANE_OPS / 1e12, 2),
            "unit": "Tops/s (vector lane-ops)",
            "frac": round(achieved / PEAK_LANE_OPS, 4),
            "frac_vs_packed_peak": round(achieved / (2 * PEAK_LANE_OPS), 4),
            "traffic": profiled_traffic(w.name),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "ops_per_launch": OPS_PER_CONTRIB * act_frac * nominal,
            "avg_launch_ms": round(das_avg_s * 1e3, 4),
        },
        "prefilter_and_qus": prefilter,
        "derivatives": derivatives,
        "pcie_inclusive": pcie,
        "paper_context": PAPER_CONTEXT,
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    if serve_summary is not None:
        res["served_stream"] = serve_summary
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
