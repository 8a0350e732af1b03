"""Pre-synthesise (and cache) the RF of named workloads with a process pool.

    python -m phantom.prepare pwi stai_full ...

Run it from a process that has not touched the GPU; later calls of
``synth_rf`` with the same workload load the cached array.
"""

import sys
import time

from .configs import get_workload
from .synth import synth_rf


def lighter(w, n_speckle=20000):
    """The same geometry with a sparser speckle field (parity sub-grid tests)."""
    a = dict(w.phantom_args)
    if "n_speckle" in a:
        a["n_speckle"] = min(a["n_speckle"], n_speckle)
    return w.with_(phantom_args=a)


def prepare(workloads, log=sys.stderr):
    for w in workloads:
        t = time.perf_counter()
        synth_rf(w)
        print(f"[phantom] {w.name} ready in {time.perf_counter() - t:.1f} s", file=log,
              flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["pwi"]
    prepare([get_workload(n) for n in names])
