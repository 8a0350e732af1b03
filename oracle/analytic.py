"""Analytic signal and envelope, FP64 (test oracle; see package docstring).

Paper: envelope detection is a post-processing op (Sec. II-B) built as the
analytic signal followed by the absolute value (Fig. 2), the analytic signal
being formed with the FFT-based Hilbert transform (Sec. II-B).  Readings: the
transform runs along depth on each image column of the beamformed RF, with
FFT length equal to the column length (no padding, hence circular), and the
standard one-sided spectrum multiplier h: h[0] = 1, h[k] = 2 for
0 < k < Z/2, h[Z/2] = 1 (even Z), 0 above.
"""

from __future__ import annotations

import numpy as np


def hilbert_multiplier(n: int) -> np.ndarray:
    """One-sided spectrum weights for an n-point analytic signal."""
    h = np.zeros(n, dtype=np.float64)
    if n == 0:
        return h
    h[0] = 1.0
    if n % 2 == 0:
        h[1 : n // 2] = 2.0
        h[n // 2] = 1.0
    else:
        h[1 : (n + 1) // 2] = 2.0
    return h


def analytic_signal(y: np.ndarray, axis: int = -2) -> np.ndarray:
    """a = IFFT(FFT(y) * h) along ``axis`` (default: depth of [..][Z][X])."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[axis]
    spec = np.fft.fft(y, axis=axis)
    shape = [1] * y.ndim
    shape[axis] = n
    return np.fft.ifft(spec * hilbert_multiplier(n).reshape(shape), axis=axis)


def envelope(y: np.ndarray, axis: int = -2) -> np.ndarray:
    """Envelope = |analytic signal| (Fig. 2: Analytic Signal -> Absolute Value)."""
    return np.abs(analytic_signal(y, axis=axis))
