"""Derivatives of Delay-and-Sum, FP64 (test oracle; see package docstring).

The paper motivates running the beamformer inside a trainable TensorFlow
graph (Sec. I; Sec. IV); the derivatives below are those of the DAS
definition in ``das.py`` (a linear map of the RF for fixed geometry):

* adjoint w.r.t. RF: for L = <g, y>, dL/dr[t, j, m] = sum over pixels p of
  w_j(p) g(p) [(1 - a) [m = n] + a [m = n + 1]], n = floor(u), a = u - n,
  only where 0 <= n <= S-2 (the transpose of the interpolating gather);
* derivative w.r.t. the speed of sound c: every time of flight is a path
  length over c, so du/dc = -(tau_tx + tau_rx) fs / c, and almost everywhere
  (away from the integer crossings of u, where the linear interpolant has a
  kink) dy(p)/dc = sum_{t, j} w_j(p) (r[n+1] - r[n]) du/dc.
"""

from __future__ import annotations

import numpy as np

from . import das as D


def das_adjoint_sum(g: np.ndarray, tau_tx: np.ndarray, tau_rx: np.ndarray, weight: np.ndarray,
                    t0: float, fs: float, n_s: int) -> np.ndarray:
    """Transpose of ``das_sum``: g [P] -> dL/drf [T][C][S]."""
    g = np.asarray(g, dtype=np.float64).ravel()
    T, C = tau_tx.shape[0], tau_rx.shape[0]
    out = np.zeros((T, C, n_s), dtype=np.float64)
    for t in range(T):
        for j in range(C):
            u = D.fractional_index(tau_tx[t].ravel(), tau_rx[j].ravel(), t0, fs)
            n = np.floor(u)
            a = u - n
            ok = (n >= 0) & (n <= n_s - 2)
            ni = n[ok].astype(np.int64)
            wg = (weight[j].ravel() * g)[ok]
            np.add.at(out[t, j], ni, (1.0 - a[ok]) * wg)
            np.add.at(out[t, j], ni + 1, a[ok] * wg)
    return out


def das_dydc_sum(rf: np.ndarray, tau_tx: np.ndarray, tau_rx: np.ndarray, weight: np.ndarray,
                 t0: float, fs: float, c: float) -> np.ndarray:
    """dy(p)/dc of ``das_sum`` (slope of the interpolant times du/dc)."""
    rf = np.asarray(rf, dtype=np.float64)
    T, C, S = rf.shape
    y = np.zeros(tau_tx.shape[1:], dtype=np.float64)
    for t in range(T):
        for j in range(C):
            u = D.fractional_index(tau_tx[t], tau_rx[j], t0, fs)
            n = np.floor(u)
            ok = (n >= 0) & (n <= S - 2)
            ni = np.where(ok, n, 0).astype(np.int64)
            slope = np.where(ok, rf[t, j, np.minimum(ni + 1, S - 1)] - rf[t, j, ni], 0.0)
            dudc = -(tau_tx[t] + tau_rx[j]) * fs / c
            y += weight[j] * slope * dudc
    return y


def _terms(w, iz=None, ix=None):
    x, z = D.workload_pixels(w, iz, ix)
    ex = D.element_positions(w.n_elem, w.pitch)
    ttx, trx = D.workload_tof(w, iz, ix)
    xr = ex[np.asarray(w.rx_elements())]
    wgt = np.stack([D.receive_weight(x, z, xe, w.f_number) for xe in xr])
    return ttx, trx, wgt


def das_adjoint_workload(g, w, iz=None, ix=None):
    """dL/drf [T][C][S] for L = <g, y> on a workload's grid (or pixels)."""
    ttx, trx, wgt = _terms(w, iz, ix)
    P = ttx.shape[1:]
    return das_adjoint_sum(np.asarray(g).reshape(P), ttx.reshape(len(ttx), -1),
                           trx.reshape(len(trx), -1), wgt.reshape(len(wgt), -1),
                           w.t0, w.fs, w.n_s)


def das_dydc_workload(rf, w, iz=None, ix=None):
    """dy/dc per pixel for a workload's grid (or pixels); rf [T][C][S]."""
    ttx, trx, wgt = _terms(w, iz, ix)
    return das_dydc_sum(rf, ttx, trx, wgt, w.t0, w.fs, w.c)
