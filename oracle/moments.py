"""Windowed moments of the envelope (qUS parametric maps), FP64 (test oracle).

Paper: the estimator use case slices the envelope of the beamformed frame and
feeds the first three moments E[X], E[X^2], E[X^3] of each slice to a network
that estimates the homodyned-K parameters (Fig. 3).  The network needs
trained weights and stays out; the moment maps are plain statistics.
Readings:

* a slice is a window of wz x wx envelope samples (depth x lateral);
* windows are placed on a regular grid with strides (sz, sx), origin
  (i sz, j sx), and only windows lying wholly inside the frame are used:
  mz = (nz - wz) // sz + 1, mx = (nx - wx) // sx + 1;
* E[X^p] is the plain mean of env^p over the window's samples, p = 1, 2, 3,
  on the linear envelope (not dB), each frame separately.

Pins: a constant envelope gives c^p; windows of a Rayleigh field match its
closed-form moments; the definition equals a brute-force scalar loop;
window placement is checked with an index ramp.
"""

from __future__ import annotations

import numpy as np


def moment_map_shape(nz: int, nx: int, wz: int, wx: int, sz: int, sx: int):
    if not (1 <= wz <= nz and 1 <= wx <= nx and sz >= 1 and sx >= 1):
        raise ValueError("window must fit the frame and strides must be positive")
    return (nz - wz) // sz + 1, (nx - wx) // sx + 1


def moment_maps(env: np.ndarray, wz: int, wx: int, sz: int, sx: int) -> np.ndarray:
    """env [F][Z][X] or [Z][X] -> maps [F][3][mz][mx] (or [3][mz][mx])."""
    e = np.asarray(env, dtype=np.float64)
    squeeze = e.ndim == 2
    if squeeze:
        e = e[None]
    n_f, nz, nx = e.shape
    mz, mx = moment_map_shape(nz, nx, wz, wx, sz, sx)
    out = np.empty((n_f, 3, mz, mx))
    inv = 1.0 / (wz * wx)
    for f in range(n_f):
        for i in range(mz):
            rows = e[f, i * sz:i * sz + wz]
            for j in range(mx):
                win = rows[:, j * sx:j * sx + wx]
                out[f, 0, i, j] = win.sum() * inv
                out[f, 1, i, j] = (win * win).sum() * inv
                out[f, 2, i, j] = (win * win * win).sum() * inv
    return out[0] if squeeze else out

