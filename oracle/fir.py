"""FIR pre-filter along the sample axis, FP64 (test oracle).

Paper: the pre-processing ops include an FIR filter applied to the raw RF
before beamforming (Sec. II-B, list of signal processing operators); no taps,
length or alignment are given.  Readings:

* every record r[f][t][c][:] (one channel of one transmit) is filtered on its
  own along samples;
* odd tap count K, output aligned to the input ("same" length and position):
  y[s] = sum_k h[k] r[s + D - k], D = (K - 1) / 2, with r = 0 outside
  [0, S) - a linear-phase filter then adds no delay, so the beamformer's
  time origin is unchanged;
* the taps are an input (any real values); the output is real RF in float.

Pins: an impulse returns the taps, a tone away from the record edges is
scaled by the moving average's Dirichlet gain, the definition equals
``numpy.convolve(..., "same")``, and edges equal the truncated sums.
"""

from __future__ import annotations

import numpy as np


def fir_same(rf: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """rf [..., S] -> filtered [..., S] (float64), y[s] = sum_k h[k] r[s+D-k]."""
    h = np.asarray(taps, dtype=np.float64)
    k_len = h.shape[0]
    if k_len % 2 != 1:
        raise ValueError("the tap count must be odd")
    r = np.asarray(rf, dtype=np.float64)
    s_len = r.shape[-1]
    d = (k_len - 1) // 2
    y = np.zeros_like(r)
    for k in range(k_len):
        shift = d - k  # y[s] += h[k] * r[s + shift]
        lo = max(0, -shift)
        hi = min(s_len, s_len - shift)
        if hi > lo:
            y[..., lo:hi] += h[k] * r[..., lo + shift:hi + shift]
    return y

