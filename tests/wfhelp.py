"""Test helpers: workload -> binding geometry, error metrics."""

import numpy as np

import paper_1811_01566_amd as wf


def scan_from_workload(w):
    g = w.grid()
    grid = wf.Grid(g["nz"], g["nx"], g["z0"], g["dz"], g["x0"], g["dx"])
    kw = dict(mode=w.mode, n_elem=w.n_elem, pitch=w.pitch, c=w.c, fs=w.fs, n_tx=w.n_tx,
              n_ch=w.n_ch, grid=grid, t0=w.t0, f_number=w.f_number,
              rx_elem=tuple(w.rx_elem) if w.rx_elem is not None else None)
    if w.mode == "stai":
        kw["tx_elem"] = tuple(w.tx_elements())
    else:
        kw["angles_rad"] = tuple(w.angles_rad())
        kw["tref"] = w.tref
    return wf.Scan(**kw)


def nl2(a, b):
    """||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
