"""Whole-frame FP64 oracle results for the full-size parity tests.

The oracle's DAS of a 1024 x 512 PWI frame (64 transmits x 128 channels)
is about 4e9 interpolate-and-adds: seconds with a process pool, a minute on
one core.  ``prepare`` computes the frames the selected tests need with a
pool forked before any GPU test initialises the device (called from
``conftest.py``) and caches them on disk, keyed by the workload and the
oracle's sources; ``das_frame`` loads them (or computes them serially when
they are missing).  Only the oracle and the seeded generator run here.
"""

from __future__ import annotations

import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import oracle
import phantom
from phantom.synth import default_workers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_RF = None  # frame-0 RF of the workload being computed (inherited by forked workers)


def _oracle_hash() -> str:
    h = hashlib.sha1()
    d = os.path.join(ROOT, "oracle")
    for name in sorted(os.listdir(d)):
        if name.endswith(".py"):
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:12]


def _path(w) -> str:
    root = os.environ.get("WF_CACHE", "/tmp/wf_cache")
    os.makedirs(root, exist_ok=True)
    key = hashlib.sha1(f"{_oracle_hash()}|{w!r}".encode()).hexdigest()[:16]
    return os.path.join(root, f"oracle_das_{w.name}_{key}.npy")


def _columns(args):
    w, c0, c1 = args
    cols = np.arange(c0, c1)
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(cols, (w.nz, 1))
    return oracle.das_workload(_RF, w, iz, ix)


def _compute(w, workers: int) -> np.ndarray:
    global _RF
    _RF = phantom.synth_rf(w)[0].astype(np.float64)
    try:
        if workers <= 1:
            return oracle.das_workload(_RF, w)
        nblk = min(w.nx, 4 * workers)
        edges = np.linspace(0, w.nx, nblk + 1).round().astype(int)
        jobs = [(w, int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]
        with ProcessPoolExecutor(max_workers=workers) as ex:
            return np.concatenate(list(ex.map(_columns, jobs)), axis=1)
    finally:
        _RF = None


def prepare(workloads, log=sys.stderr) -> None:
    """Compute and cache the frame-0 oracle DAS of each workload (run from a
    process that has not initialised a GPU, so that a pool may be forked)."""
    workers = default_workers()
    for w in workloads:
        p = _path(w)
        if os.path.exists(p):
            continue
        t = time.perf_counter()
        y = _compute(w, workers)
        tmp = p + f".tmp{os.getpid()}.npy"
        np.save(tmp, y)
        os.replace(tmp, p)
        print(f"[oracle] {w.name}: whole frame in {time.perf_counter() - t:.1f} s "
              f"({workers} workers)", file=log, flush=True)


def das_frame(w) -> np.ndarray:
    """The oracle's DAS of frame 0 of workload w, [nz][nx] float64."""
    p = _path(w)
    if os.path.exists(p):
        return np.load(p, allow_pickle=False)
    prepare([w])
    return np.load(p, allow_pickle=False)


def served_test_pool():
    """The shape classes the served-stream GPU test draws its requests from:
    speckle + cyst phantoms of the served mix."""
    from phantom.configs import served_pool

    return list(served_pool(8, seed=11))


# workloads whose whole-frame oracle a test marked ``oracle_frames(name)`` needs
FRAME_SETS = {
    "pwi": lambda: [phantom.get_workload("pwi")],
    "stai_full": lambda: [phantom.get_workload("stai_full")],
    "served": served_test_pool,
}
