"""Log compression and dynamic-range clipping, FP64 (test oracle).

Paper: "dynamic adjustment" is the last op of the B-mode pipeline (Fig. 2;
Sec. II-B) and the evaluation clips the frame to [0, 30] dB (Sec. III).
Readings: amplitude dB, B = 20 log10(env / m) with m the maximum envelope of
the frame (each frame of a batch separately), clipped to [-DR, 0]; a zero
envelope or an all-zero frame maps to -DR (never NaN or -inf); with
``offset`` the result is shifted by +DR into [0, DR] as in the paper's
display range.
"""

from __future__ import annotations

import numpy as np


def log_compress(env: np.ndarray, dr_db: float, offset: bool = False) -> np.ndarray:
    """env [F][Z][X] or [Z][X] -> dB image, per-frame reference."""
    env = np.asarray(env, dtype=np.float64)
    squeeze = env.ndim == 2
    e = env[None] if squeeze else env
    out = np.empty_like(e)
    for f in range(e.shape[0]):
        m = float(e[f].max()) if e[f].size else 0.0
        if m <= 0.0:
            out[f] = -dr_db
            continue
        with np.errstate(divide="ignore"):
            b = 20.0 * np.log10(e[f] / m)
        b = np.where(e[f] > 0, b, -dr_db)
        out[f] = np.clip(b, -dr_db, 0.0)
    if offset:
        out = out + dr_db
    return out[0] if squeeze else out


def bmode(y: np.ndarray, dr_db: float, offset: bool = False) -> np.ndarray:
    """Beamformed RF -> B-mode frame: envelope then log compression (Fig. 2)."""
    from .analytic import envelope

    return log_compress(envelope(y), dr_db, offset)
