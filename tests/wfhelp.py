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


def deep_pwi():
    """A PWI grid reaching deeper than its record (512 samples, 1-12 mm):
    the lower tiles receive no echo, so the DAS work split leaves them out
    of its work list."""
    import numpy as np

    import phantom

    return phantom.tiny_pwi(name="deep_pwi", n_elem=32, n_tx=8, n_ch=32, n_s=512, nz=256,
                            nx=64, z_min=1e-3, z_max=12e-3,
                            angles_deg=tuple(float(a) for a in np.linspace(-10.0, 10.0, 8)))
