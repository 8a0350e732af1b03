"""FIR taps for the pre-filter workloads (inputs, not the method).

The paper's pre-processing FIR (Sec. II-B) comes with no taps; the workloads
use a linear-phase band-pass around the transmit frequency: the difference
of two ideal low-pass impulse responses (windowed sinc) under a Hamming
window, rounded to float32 so that the oracle and the kernels consume the
same values.
"""

from __future__ import annotations

import numpy as np


def bandpass_taps(n_taps: int, f_lo: float, f_hi: float, fs: float) -> np.ndarray:
    if n_taps % 2 != 1 or n_taps < 1:
        raise ValueError("n_taps must be odd and positive")
    if not 0.0 <= f_lo < f_hi <= fs / 2:
        raise ValueError("need 0 <= f_lo < f_hi <= fs / 2")
    m = np.arange(n_taps) - (n_taps - 1) / 2.0
    ideal = 2.0 * f_hi / fs * np.sinc(2.0 * f_hi / fs * m) - 2.0 * f_lo / fs * np.sinc(
        2.0 * f_lo / fs * m)
    win = 0.54 - 0.46 * np.cos(2.0 * np.pi * np.arange(n_taps) / max(1, n_taps - 1))
    return (ideal * win).astype(np.float32)


def workload_taps(w, n_taps: int = 31) -> np.ndarray:
    """Band-pass [0.5 fc, 1.5 fc] (fc = the workload's pulse centre frequency)."""
    return bandpass_taps(n_taps, 0.5 * w.fc, 1.5 * w.fc, w.fs)
