"""Delay-and-Sum beamforming, FP64 (test oracle; see package docstring).

Paper: DAS is the mid-processing op, with STAI and PWI variants (Sec. II-B);
its input is the RF tensor (acquisitions, channels, samples) plus metadata -
speed of sound, aperture, sampling frequency (Sec. II-A; Sec. III).  The
paper gives no formula; the readings used here:

* linear array on z = 0, element e at x_e = (e - (N-1)/2) pitch, or an
  explicit list; omnidirectional point elements;
* receive time of flight  tau_rx = |p - e_j| / c;
* STAI transmit t (single element e_t)  tau_tx = |p - e_t| / c;
* PWI transmit k at angle theta_k (> 0 steers towards +x)
  tau_tx = (z cos theta_k + x sin theta_k + o_k) / c, with
  o_k = -min_e(x_e sin theta_k) when time zero is the firing of the first
  element ("first"), o_k = 0 when it is the wavefront crossing x = 0 ("centre");
* fractional sample index u = (tau_tx + tau_rx - t0) fs, sample s recorded
  at t0 + s / fs;
* linear interpolation between r[n] and r[n+1], n = floor(u); the
  contribution is 0 unless 0 <= n <= S-2;
* receive apodisation: boxcar w_j(p) = 1 iff 2 F# |x - x_j| <= z (F# > 0),
  else w = 1; no transmit apodisation, no normalisation;
* y(p) = sum over transmits t and channels j of w_j(p) v_{t,j}(p); PWI
  compounding is this same unweighted sum over angles.
"""

from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np


def element_positions(n_elem: int, pitch: float, elem_x=None) -> np.ndarray:
    """Lateral element positions (m): centred uniform linear array unless
    given explicitly.  Reading of the 'aperture size' metadata (Sec. II-A)."""
    if elem_x is not None:
        return np.asarray(elem_x, dtype=np.float64)
    e = np.arange(n_elem, dtype=np.float64)
    return (e - (n_elem - 1) / 2.0) * pitch


def pixel_positions(nz: int, nx: int, z0: float, dz: float, x0: float, dx: float):
    """(x, z) of every pixel of the [nz][nx] grid, depth-major (the paper's
    output frames are (depth samples, lines), Sec. III)."""
    iz = np.arange(nz, dtype=np.float64)[:, None]
    ix = np.arange(nx, dtype=np.float64)[None, :]
    x = np.broadcast_to(x0 + ix * dx, (nz, nx))
    z = np.broadcast_to(z0 + iz * dz, (nz, nx))
    return np.ascontiguousarray(x), np.ascontiguousarray(z)


def tof_receive(x, z, x_elem: float, c: float):
    """Receive time of flight from pixel (x, z) to an element at (x_elem, 0)."""
    return np.sqrt((np.asarray(x) - x_elem) ** 2 + np.asarray(z) ** 2) / c


def tof_stai_transmit(x, z, x_elem: float, c: float):
    """STAI: a single element at (x_elem, 0) fires; spherical wave to (x, z)."""
    return np.sqrt((np.asarray(x) - x_elem) ** 2 + np.asarray(z) ** 2) / c


def pwi_time_offset(theta: float, elem_x: np.ndarray, tref: str) -> float:
    """Distance term o_k of a plane-wave transmit (m).  'first': time zero
    when the first element fires, so o_k = -min_e(x_e sin theta); 'centre':
    time zero when the wavefront crosses the array centre, o_k = 0."""
    if tref == "centre":
        return 0.0
    if tref != "first":
        raise ValueError(tref)
    return float(-np.min(np.asarray(elem_x) * math.sin(theta)))


def tof_pwi_transmit(x, z, theta: float, elem_x: np.ndarray, c: float,
                     tref: str = "first"):
    """PWI: plane wave steered by theta (> 0 towards +x)."""
    o = pwi_time_offset(theta, elem_x, tref)
    return (np.asarray(z) * math.cos(theta) + np.asarray(x) * math.sin(theta) + o) / c


def fractional_index(tau_tx, tau_rx, t0: float, fs: float):
    """u = (tau_tx + tau_rx - t0) * fs: position of the echo in the record."""
    return (np.asarray(tau_tx) + np.asarray(tau_rx) - t0) * fs


def interp_linear(row: np.ndarray, u) -> np.ndarray:
    """Linear interpolation of one RF row at fractional sample u; 0 unless
    0 <= floor(u) <= S-2."""
    u = np.asarray(u, dtype=np.float64)
    s = row.shape[0]
    n = np.floor(u)
    a = u - n
    ok = (n >= 0) & (n <= s - 2)
    ni = np.where(ok, n, 0).astype(np.int64)
    v = (1.0 - a) * row[ni] + a * row[np.minimum(ni + 1, s - 1)]
    return np.where(ok, v, 0.0)


def receive_weight(x, z, x_elem: float, f_number: float):
    """Receive apodisation: boxcar aperture of f-number F# (inclusive edge);
    all ones when F# <= 0."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if f_number <= 0:
        return np.ones(np.broadcast(x, z).shape)
    return (2.0 * f_number * np.abs(x - x_elem) <= z).astype(np.float64)


def das_sum(rf: np.ndarray, tau_tx: np.ndarray, tau_rx: np.ndarray,
            weight: np.ndarray, t0: float, fs: float) -> np.ndarray:
    """y(p) = sum_t sum_j w_j(p) * lerp(rf[t, j], u_tj(p)).

    rf [T][C][S]; tau_tx [T][P]; tau_rx [C][P]; weight [C][P] -> y [P]."""
    rf = np.asarray(rf, dtype=np.float64)
    T, C, _ = rf.shape
    y = np.zeros(tau_tx.shape[1:], dtype=np.float64)
    for t in range(T):
        for j in range(C):
            u = fractional_index(tau_tx[t], tau_rx[j], t0, fs)
            y += weight[j] * interp_linear(rf[t, j], u)
    return y


def _rx_terms(x, z, elem_x, rx_elem, c, f_number):
    xr = elem_x[np.asarray(rx_elem)]
    tau_rx = np.stack([tof_receive(x, z, xe, c) for xe in xr])
    w = np.stack([receive_weight(x, z, xe, f_number) for xe in xr])
    return tau_rx, w


def das_stai(rf, x, z, elem_x, tx_elem: Sequence[int], rx_elem: Sequence[int],
             c: float, fs: float, t0: float = 0.0, f_number: float = 0.0):
    """STAI Delay-and-Sum (Sec. II-B) at pixel positions x, z (any shape).
    rf [T][C][S] or [F][T][C][S]."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    elem_x = np.asarray(elem_x, dtype=np.float64)
    tau_tx = np.stack([tof_stai_transmit(x, z, elem_x[e], c) for e in tx_elem])
    tau_rx, w = _rx_terms(x, z, elem_x, rx_elem, c, f_number)
    rf = np.asarray(rf)
    if rf.ndim == 4:
        return np.stack([das_sum(r, tau_tx, tau_rx, w, t0, fs) for r in rf])
    return das_sum(rf, tau_tx, tau_rx, w, t0, fs)


def das_pwi(rf, x, z, elem_x, angles: Sequence[float], rx_elem: Sequence[int],
            c: float, fs: float, t0: float = 0.0, f_number: float = 0.0,
            tref: str = "first"):
    """PWI Delay-and-Sum with coherent compounding over angles (Sec. II-B)."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    elem_x = np.asarray(elem_x, dtype=np.float64)
    tau_tx = np.stack([tof_pwi_transmit(x, z, th, elem_x, c, tref) for th in angles])
    tau_rx, w = _rx_terms(x, z, elem_x, rx_elem, c, f_number)
    rf = np.asarray(rf)
    if rf.ndim == 4:
        return np.stack([das_sum(r, tau_tx, tau_rx, w, t0, fs) for r in rf])
    return das_sum(rf, tau_tx, tau_rx, w, t0, fs)


def workload_pixels(w, iz=None, ix=None):
    g = w.grid()
    x, z = pixel_positions(g["nz"], g["nx"], g["z0"], g["dz"], g["x0"], g["dx"])
    if iz is not None:
        return x[iz, ix], z[iz, ix]
    return x, z


def das_workload(rf, w, iz=None, ix=None, x=None, z=None):
    """DAS of a ``phantom.Workload`` on its whole grid, or on the pixels
    (iz, ix) (index arrays of equal shape), or on explicit positions."""
    if x is None:
        x, z = workload_pixels(w, iz, ix)
    ex = element_positions(w.n_elem, w.pitch)
    common = dict(c=w.c, fs=w.fs, t0=w.t0, f_number=w.f_number)
    if w.mode == "stai":
        return das_stai(rf, x, z, ex, w.tx_elements(), w.rx_elements(), **common)
    return das_pwi(rf, x, z, ex, w.angles_rad(), w.rx_elements(), tref=w.tref, **common)


def workload_tof(w, iz=None, ix=None):
    """(tau_tx [T][...], tau_rx [C][...]) in seconds for a workload's pixels."""
    x, z = workload_pixels(w, iz, ix)
    ex = element_positions(w.n_elem, w.pitch)
    if w.mode == "stai":
        ttx = np.stack([tof_stai_transmit(x, z, ex[e], w.c) for e in w.tx_elements()])
    else:
        ttx = np.stack([tof_pwi_transmit(x, z, th, ex, w.c, w.tref) for th in w.angles_rad()])
    trx = np.stack([tof_receive(x, z, ex[e], w.c) for e in w.rx_elements()])
    return ttx, trx
