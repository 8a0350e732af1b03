"""Forward acoustic model: point scatterers -> int16 RF channel data.

Model (readings; the paper gives no simulation model, its data were measured):

* pulse p(t) = exp(-t^2 / (2 sigma^2)) * cos(2 pi fc t + phi), with a Gaussian
  envelope whose full width at half maximum is two carrier periods, i.e.
  sigma = 2 / (fc * 2 sqrt(2 ln 2));
* an echo from a scatterer of complex amplitude a = |a| e^{i phi} at (x, z)
  is Re[a * P(t - tau)], P the analytic pulse, tau = transmit time of flight
  + receive time of flight, omnidirectional elements, no attenuation;
* white Gaussian noise at the requested SNR (noise sigma = 10^(-SNR/20) x RMS
  of the noiseless record of the whole frame);
* int16 quantisation: scaled so that max |rf| = 8191 (14-bit full scale),
  rounded half to even, clipped to +-32767.

Sparse phantoms are synthesised with exact analytic pulses.  Dense speckle
uses complex-amplitude time histograms at 16x the sampling rate (carrier
phase corrected to the exact arrival time) convolved with the analytic pulse.

The time-of-flight code here is the generator's own: it is written
independently of the beamformer's so that a focusing test is not a test of
one formula against itself.
"""

from __future__ import annotations

import hashlib
import math
import os
from concurrent.futures import ProcessPoolExecutor
from typing import Optional, Sequence, Tuple

import numpy as np

from .configs import Workload

GEN_VERSION = 4
UPSAMPLE = 16
ADC_FULL_SCALE = 8191.0


def pulse_sigma(fc: float) -> float:
    return 2.0 / (fc * 2.0 * math.sqrt(2.0 * math.log(2.0)))


def _first_firing_x(elem_x: np.ndarray, theta: float, tref: str) -> float:
    if tref == "centre":
        return 0.0
    return float(elem_x.min() if math.sin(theta) >= 0 else elem_x.max())


def _tx_times(w: Workload, xs: np.ndarray, zs: np.ndarray, t: int) -> np.ndarray:
    """Transmit time of flight of transmit t to each scatterer (s)."""
    ex = np.asarray(w.elem_x(), dtype=np.float64)
    if w.mode == "stai":
        e = w.tx_elements()[t]
        return np.hypot(xs - ex[e], zs) / w.c
    th = w.angles_rad()[t]
    xf = _first_firing_x(ex, th, w.tref)
    # plane wave leaving the first-firing element (xf, 0) at t = 0
    return ((xs - xf) * math.sin(th) + zs * math.cos(th)) / w.c


def _rx_times(w: Workload, xs: np.ndarray, zs: np.ndarray) -> np.ndarray:
    ex = np.asarray(w.elem_x(), dtype=np.float64)[w.rx_elements()]
    return np.hypot(xs[None, :] - ex[:, None], zs[None, :]) / w.c  # [C, K]


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

def scatterers_for(w: Workload, frame: int = 0):
    """(x, z, a) arrays of the phantom for one frame; a is complex."""
    rng = np.random.default_rng(np.random.SeedSequence([w.seed, frame]))
    ex = w.elem_x()
    xa, xb = ex[0], ex[-1]
    args = w.phantom_args
    if w.phantom == "points_on_pixels":
        g = w.grid()
        pts = args["pixels"]
        xs = np.array([g["x0"] + ix * g["dx"] for (_, ix) in pts])
        zs = np.array([g["z0"] + iz * g["dz"] for (iz, _) in pts])
        return xs, zs, np.ones(len(pts), dtype=np.complex128)
    if w.phantom == "points":
        xs = np.asarray(args["x"], dtype=np.float64)
        zs = np.asarray(args["z"], dtype=np.float64)
        a = np.asarray(args.get("a", np.ones(len(xs))), dtype=np.complex128)
        return xs, zs, a
    if w.phantom == "wires_speckle":
        wx, wz = np.meshgrid(np.asarray(args["wires_x_mm"]) * 1e-3,
                             np.asarray(args["wires_z_mm"]) * 1e-3)
        n = int(args["n_speckle"])
        z0, z1 = args["z_range_mm"]
        sx = rng.uniform(xa, xb, n)
        sz = rng.uniform(z0 * 1e-3, z1 * 1e-3, n)
        sa = rng.normal(0.0, args["speckle_sigma"], n)
        xs = np.concatenate([wx.ravel(), sx])
        zs = np.concatenate([wz.ravel(), sz])
        a = np.concatenate([np.ones(wx.size), sa]).astype(np.complex128)
        return xs, zs, a
    if w.phantom == "cysts":
        n = int(args["n_speckle"])
        z0, z1 = args["z_range_mm"]
        sx = rng.uniform(xa, xb, n)
        sz = rng.uniform(z0 * 1e-3, z1 * 1e-3, n)
        # Rayleigh(1) magnitude with uniform phase
        mag = rng.rayleigh(1.0, n)
        ph = rng.uniform(0.0, 2 * math.pi, n)
        keep = np.ones(n, dtype=bool)
        r = args["cyst_radius_mm"] * 1e-3
        for (cx, cz) in args["cysts_mm"]:
            keep &= np.hypot(sx - cx * 1e-3, sz - cz * 1e-3) > r
        return sx[keep], sz[keep], (mag * np.exp(1j * ph))[keep]
    raise ValueError(f"unknown phantom {w.phantom!r}")


# --------------------------------------------------------------------------
# exact analytic synthesis (sparse scatterers)
# --------------------------------------------------------------------------

def _exact_tx(w: Workload, xs, zs, a, t: int) -> np.ndarray:
    sig = pulse_sigma(w.fc)
    half = int(math.ceil(8 * sig * w.fs)) + 1
    tau = _tx_times(w, xs, zs, t)[None, :] + _rx_times(w, xs, zs)  # [C, K]
    out = np.zeros((w.n_ch, w.n_s), dtype=np.float64)
    centre = (tau - w.t0) * w.fs  # fractional sample of arrival
    offs = np.arange(-half, half + 1)
    for c in range(w.n_ch):
        s = np.floor(centre[c])[:, None].astype(np.int64) + offs[None, :]  # [K, L]
        tt = (w.t0 + s / w.fs) - tau[c][:, None]
        v = np.real(a[:, None] * np.exp(-tt * tt / (2 * sig * sig))
                    * np.exp(2j * math.pi * w.fc * tt))
        ok = (s >= 0) & (s < w.n_s)
        out[c] = np.bincount(s[ok], weights=v[ok], minlength=w.n_s)[: w.n_s]
    return out


# --------------------------------------------------------------------------
# histogram synthesis (dense speckle)
# --------------------------------------------------------------------------

def _smooth_len(n: int) -> int:
    """Smallest 2^a 3^b 5^c >= n (a fast FFT length)."""
    best = 1 << int(math.ceil(math.log2(n)))
    p5 = 1
    while p5 < best:
        p35 = p5
        while p35 < best:
            m = p35
            while m < n:
                m *= 2
            best = min(best, m)
            p35 *= 3
        p5 *= 5
    return best


def _kernel_fft(w: Workload, nfft: int, margin: int) -> np.ndarray:
    sig = pulse_sigma(w.fc)
    k = np.arange(-margin, margin + 1)
    tk = k / (w.fs * UPSAMPLE)
    ker = np.exp(-tk * tk / (2 * sig * sig)) * np.exp(2j * math.pi * w.fc * tk)
    buf = np.zeros(nfft, dtype=np.complex128)
    buf[: ker.size] = ker
    return np.fft.fft(buf)


def _hist_tx(w: Workload, xs, zs, a, t: int, chunk: int = 16) -> np.ndarray:
    sig = pulse_sigma(w.fc)
    margin = int(math.ceil(8 * sig * w.fs * UPSAMPLE)) + 1
    L = w.n_s * UPSAMPLE + 2 * margin  # histogram support incl. leakage margin
    nfft = _smooth_len(L + 2 * margin + 1)
    kf = _kernel_fft(w, nfft, margin)
    ttx = _tx_times(w, xs, zs, t)
    ex = np.asarray(w.elem_x(), dtype=np.float64)[w.rx_elements()]
    out = np.zeros((w.n_ch, w.n_s), dtype=np.float64)
    for c0 in range(0, w.n_ch, chunk):
        cs = slice(c0, min(c0 + chunk, w.n_ch))
        nc = cs.stop - cs.start
        tau = ttx[None, :] + np.hypot(xs[None, :] - ex[cs, None], zs[None, :]) / w.c
        q = (tau - w.t0) * (w.fs * UPSAMPLE)
        b = np.rint(q)
        delta = (q - b) / (w.fs * UPSAMPLE)
        wgt = a[None, :] * np.exp(-2j * math.pi * w.fc * delta)
        bi = b.astype(np.int64) + margin
        ok = (bi >= 0) & (bi < L)
        flat = (np.arange(nc)[:, None] * L + bi)[ok]
        hr = np.bincount(flat, weights=wgt.real[ok], minlength=nc * L)
        hi = np.bincount(flat, weights=wgt.imag[ok], minlength=nc * L)
        h = np.zeros((nc, nfft), dtype=np.complex128)
        h[:, :L] = (hr + 1j * hi).reshape(nc, L)
        conv = np.fft.ifft(np.fft.fft(h, axis=1) * kf[None, :], axis=1)
        # output sample s sits at histogram bin s*U + margin, kernel centre
        # at index margin of the kernel buffer
        idx = np.arange(w.n_s) * UPSAMPLE + 2 * margin
        out[cs] = conv[:, idx].real
    return out


def _synth_tx_block(args):
    w, xs, zs, a, ts, exact = args
    fn = _exact_tx if exact else _hist_tx
    return np.stack([fn(w, xs, zs, a, t) for t in ts])


def _frame_float(w: Workload, frame: int, workers: int) -> np.ndarray:
    xs, zs, a = scatterers_for(w, frame)
    exact = xs.size <= 256
    ts = list(range(w.n_tx))
    if workers <= 1 or w.n_tx < 2:
        return _synth_tx_block((w, xs, zs, a, ts, exact))
    blocks = [ts[i::workers] for i in range(workers) if ts[i::workers]]
    out = np.zeros((w.n_tx, w.n_ch, w.n_s), dtype=np.float64)
    with ProcessPoolExecutor(max_workers=len(blocks)) as ex:
        for blk, res in zip(blocks, ex.map(_synth_tx_block,
                                           [(w, xs, zs, a, b, exact) for b in blocks])):
            out[blk] = res
    return out


def _cache_path(w: Workload, tag: str) -> Optional[str]:
    root = os.environ.get("WF_CACHE", "/tmp/wf_cache")
    try:
        os.makedirs(root, exist_ok=True)
    except OSError:
        return None
    key = hashlib.sha1(f"{GEN_VERSION}|{tag}|{w!r}".encode()).hexdigest()[:16]
    return os.path.join(root, f"{w.name}_{tag}_{key}.npy")


def _gpu_initialised() -> bool:
    import sys

    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:  # pragma: no cover
        return True


def default_workers() -> int:
    """Worker processes for synthesis: up to 16, and none once this process
    has initialised a GPU (worker pools are only forked from clean processes)."""
    if _gpu_initialised():
        return 1
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def synth_rf(w: Workload, quantize: bool = True, workers: Optional[int] = None,
             cache: bool = True, frames: Optional[Sequence[int]] = None) -> np.ndarray:
    """RF channel data [F][T][C][S]: int16 counts (quantize=True) or the
    pre-quantisation record in the same count units (float64; cached as
    float32, i.e. to ~1e-7 relative).  One synthesis fills both caches."""
    frames = list(range(w.n_frames)) if frames is None else list(frames)
    if w.phantom == "random":
        rng = np.random.default_rng(np.random.SeedSequence([w.seed, 99]))
        r = rng.integers(-8191, 8192, size=(len(frames), w.n_tx, w.n_ch, w.n_s))
        return r.astype(np.int16 if quantize else np.float64)
    fkey = "-".join(map(str, frames))
    p16 = _cache_path(w, "i16_" + fkey) if cache else None
    p32 = _cache_path(w, "f32_" + fkey) if cache else None
    want = p16 if quantize else p32
    if want and os.path.exists(want):
        arr = np.load(want, allow_pickle=False)
        return arr if quantize else arr.astype(np.float64)
    workers = default_workers() if workers is None else min(workers, default_workers())
    q, raw = [], []
    for f in frames:
        rf = _frame_float(w, f, workers)
        if w.snr_db is not None:
            rng = np.random.default_rng(np.random.SeedSequence([w.seed, f, 7]))
            rms = math.sqrt(float(np.mean(rf * rf)))
            rf = rf + rng.normal(0.0, rms * 10.0 ** (-w.snr_db / 20.0), rf.shape)
        peak = float(np.max(np.abs(rf)))
        scale = ADC_FULL_SCALE / peak if peak > 0 else 1.0
        rf = rf * scale
        q.append(np.clip(np.rint(rf), -32767, 32767).astype(np.int16))
        raw.append(rf.astype(np.float32) if cache else rf)
    a16 = np.stack(q)
    a32 = np.stack(raw)
    for path, arr in ((p16, a16), (p32, a32)):
        if path:
            tmp = path + f".tmp{os.getpid()}.npy"
            np.save(tmp, arr)
            os.replace(tmp, path)
    return a16 if quantize else a32.astype(np.float64)


def point_echo_rf(w: Workload, x: float, z: float, amp: complex = 1.0) -> np.ndarray:
    """Noiseless float64 RF [T][C][S] of one point scatterer (exact pulses)."""
    xs = np.array([x]); zs = np.array([z]); a = np.array([amp], dtype=np.complex128)
    return np.stack([_exact_tx(w, xs, zs, a, t) for t in range(w.n_tx)])
