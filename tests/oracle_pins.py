"""Pins of the FP64 oracle against facts the mathematics fixes.

Each ``pin_*`` raises AssertionError when the oracle disagrees with a closed
form, an invariant or a brute-force evaluation on a tiny input.  They are
collected by ``test_oracle_pins.py`` and re-run against deliberately broken
oracles by ``test_oracle_mutations.py`` (every planted mistake must make at
least one pin fail).  Functions are reached through the oracle submodules so
that a monkeypatched step is seen by the functions that use it.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np

import phantom
import phantom.synth
from oracle import dbclip as B
from oracle import das as D
from oracle import adjoint as A
from oracle import analytic as E
from oracle import fir as F
from oracle import moments as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _close(a, b, rtol=1e-12, atol=0.0, msg=""):
    a = np.asarray(a)
    b = np.asarray(b)
    if not (np.iscomplexobj(a) or np.iscomplexobj(b)):
        a = a.astype(np.float64)
        b = b.astype(np.float64)
    if not np.allclose(a, b, rtol=rtol, atol=atol):
        err = np.max(np.abs(a - b))
        raise AssertionError(f"{msg}: max abs diff {err:.3e}")


# --------------------------------------------------------------------------
# times of flight (DAS geometry, Sec. II-A metadata / Sec. II-B DAS)
# --------------------------------------------------------------------------

def pin_tof_golden():
    g = json.load(open(os.path.join(GOLDEN, "tof_closed_form.json")))
    c = g["c"]
    for case in g["cases"]:
        k = case["kind"]
        if k == "receive":
            got = D.tof_receive(case["x"], case["z"], case["x_elem"], c)
        elif k == "stai_transmit":
            got = D.tof_stai_transmit(case["x"], case["z"], case["x_elem"], c)
        else:
            ex = D.element_positions(case["n_elem"], case["pitch"])
            got = D.tof_pwi_transmit(case["x"], case["z"], math.radians(case["theta_deg"]),
                                     ex, c, case["tref"])
        _close(got, case["tau"], rtol=1e-12, atol=1e-20, msg=f"tof {case['note']}")


def pin_pwi_wavefront_geometry():
    """A plane wave steered by theta travels along (sin theta, cos theta):
    moving a distance d along that direction adds d / c, moving along the
    wavefront adds nothing; the first-firing element sees time 0."""
    c = 1540.0
    ex = D.element_positions(16, 0.3e-3)
    for deg in (-20.0, -7.5, 4.0, 16.0):
        th = math.radians(deg)
        x, z = 1.3e-3, 9.0e-3
        t0 = D.tof_pwi_transmit(x, z, th, ex, c, "first")
        d = 2.5e-3
        t_prop = D.tof_pwi_transmit(x + d * math.sin(th), z + d * math.cos(th), th, ex, c, "first")
        t_front = D.tof_pwi_transmit(x + d * math.cos(th), z - d * math.sin(th), th, ex, c, "first")
        _close(t_prop - t0, d / c, rtol=1e-10, msg="propagation direction")
        _close(t_front, t0, rtol=1e-10, msg="along the wavefront")
        first = ex[0] if th > 0 else ex[-1]
        _close(D.tof_pwi_transmit(first, 0.0, th, ex, c, "first"), 0.0, atol=1e-20,
               msg="first element fires at t = 0")
        # every element is reached at or after time 0
        assert np.all(D.tof_pwi_transmit(ex, np.zeros_like(ex), th, ex, c, "first") >= -1e-18)


# --------------------------------------------------------------------------
# gather / interpolate / accumulate
# --------------------------------------------------------------------------

def _deep_stai(n=8, s=4096, f_number=0.0):
    # record long enough that every pixel's echo is inside the window
    return phantom.tiny_stai(n_elem=n, n_tx=n, n_ch=n, n_s=s, nz=5, nx=7,
                             z_min=4e-3, z_max=12e-3, f_number=f_number)


def pin_constant_rf_counts():
    """RF = 1 everywhere: each active (transmit, channel) pair adds exactly 1."""
    w = _deep_stai()
    rf = np.ones((w.n_tx, w.n_ch, w.n_s))
    y = D.das_workload(rf, w)
    _close(y, np.full(y.shape, w.n_tx * w.n_ch), rtol=0, atol=1e-9, msg="all active")
    # f-number aperture: pixel straight below element 3 at the depth where
    # the half-aperture z / (2 F#) is 2.5 pitches -> elements 1..5 active
    pitch = w.pitch
    fnum = 1.5
    ex = D.element_positions(w.n_elem, pitch)
    z = 2 * fnum * 2.5 * pitch
    y1 = D.das_stai(rf, np.array([ex[3]]), np.array([z]), ex, range(w.n_tx), range(w.n_ch),
                    w.c, w.fs, f_number=fnum)
    _close(y1, [w.n_tx * 5], rtol=0, atol=1e-9, msg="f-number aperture count")
    # pixel whose echoes all arrive after the record ends -> nothing
    deep = (w.n_s + 10) / w.fs * w.c / 2
    y2 = D.das_stai(rf, np.array([0.0]), np.array([deep]), ex, range(w.n_tx), range(w.n_ch),
                    w.c, w.fs)
    _close(y2, [0.0], rtol=0, atol=0, msg="beyond the record")


def pin_linear_ramp():
    """r[s] = a + b s is reproduced exactly by linear interpolation, so
    y = sum over pairs of (a + b u) with u = (tau_tx + tau_rx - t0) fs."""
    a, b = 3.0, 0.25
    for mode in ("stai", "pwi"):
        w = _deep_stai() if mode == "stai" else phantom.tiny_pwi(
            n_elem=8, n_ch=8, n_s=4096, nz=5, nx=7, z_min=4e-3, z_max=12e-3,
            angles_deg=(-11.0, 0.0, 6.0))
        w = w.with_(t0=0.7e-6)
        rf = np.broadcast_to(a + b * np.arange(w.n_s, dtype=np.float64),
                             (w.n_tx, w.n_ch, w.n_s))
        y = D.das_workload(rf, w)
        g = w.grid()
        ex = [(e - (w.n_elem - 1) / 2) * w.pitch for e in range(w.n_elem)]
        exp = np.zeros((w.nz, w.nx))
        for iz in range(w.nz):
            for ix in range(w.nx):
                x = g["x0"] + ix * g["dx"]
                z = g["z0"] + iz * g["dz"]
                if mode == "stai":
                    ttx = [math.hypot(x - ex[e], z) / w.c for e in w.tx_elements()]
                else:
                    ttx = []
                    for th in w.angles_rad():
                        # first element to fire is the one the wave leaves first
                        xf = ex[0] if th >= 0 else ex[-1]
                        ttx.append(((x - xf) * math.sin(th) + z * math.cos(th)) / w.c)
                trx = [math.hypot(x - ex[j], z) / w.c for j in w.rx_elements()]
                tot = 0.0
                for tt in ttx:
                    for tr in trx:
                        tot += a + b * (tt + tr - w.t0) * w.fs
                exp[iz, ix] = tot
        _close(y, exp, rtol=1e-11, msg=f"linear ramp {mode}")


def pin_window_edges():
    """One element, one transmit, pixel straight below it: u = 2 z fs / c - t0 fs.
    With a ramp r[s] = a + b s the contribution is a + b u exactly when
    0 <= floor(u) <= S-2 and 0 otherwise."""
    a, b = -2.0, 0.5
    c, fs, S = 1500.0, 40e6, 256
    rf = (a + b * np.arange(S, dtype=np.float64))[None, None, :]
    ex = np.array([0.0])
    cases = [(S - 1.5, a + b * (S - 1.5)), (S - 2.0, a + b * (S - 2.0)), (S - 0.75, 0.0),
             (S + 3.0, 0.0), (0.25, a + b * 0.25), (0.0, a), (-0.5, 0.0)]
    for t0 in (0.0, 0.4e-6):
        for u, expect in cases:
            z = (u + t0 * fs) * c / (2 * fs)
            if z < 0:
                continue
            y = D.das_stai(rf, np.array([0.0]), np.array([z]), ex, [0], [0], c, fs, t0=t0)
            _close(y, [expect], rtol=1e-12, atol=1e-12, msg=f"window edge u={u} t0={t0}")


def _scatterer_workload(mode):
    common = dict(n_elem=16, n_ch=16, pitch=0.3e-3, fc=5e6, fs=50e6, c=1540.0, n_s=1024,
                  nz=41, nx=31, z_min=6e-3, z_max=10e-3)
    if mode == "stai":
        return phantom.tiny_stai(n_tx=16, **common)
    return phantom.tiny_pwi(n_tx=5, angles_deg=(-10.0, -4.0, 0.0, 5.0, 12.0), **common)


def pin_point_scatterer_focus():
    """A noiseless point echo (generator's own forward model) focuses at its
    pixel, with a normalised peak close to 1 (bounds below)."""
    for mode in ("stai", "pwi"):
        w = _scatterer_workload(mode)
        g = w.grid()
        iz, ix = 23, 12
        x = g["x0"] + ix * g["dx"]
        z = g["z0"] + iz * g["dz"]
        rf = phantom.point_echo_rf(w, x, z)
        y = D.das_workload(rf, w)
        env = E.envelope(y)
        k = np.unravel_index(np.argmax(env), env.shape)
        assert k == (iz, ix), f"{mode}: focus at {k}, scatterer at {(iz, ix)}"
        peak = y[iz, ix] / (w.n_tx * w.n_ch)
        # each pair samples the pulse at most one sample from its peak:
        # lerp of the carrier loses at most cos(pi fc / fs), the Gaussian
        # envelope at most exp(-1 / (2 sigma^2))
        sig = phantom.synth.pulse_sigma(w.fc) * w.fs
        lo = math.cos(math.pi * w.fc / w.fs) * math.exp(-1.0 / (2 * sig * sig))
        assert lo - 1e-9 <= peak <= 1 + 1e-9, f"{mode}: normalised peak {peak}"


def pin_linearity():
    w = phantom.tiny_pwi(f_number=1.0)
    rng = np.random.default_rng(5)
    r1 = rng.normal(size=(w.n_tx, w.n_ch, w.n_s))
    r2 = rng.normal(size=(w.n_tx, w.n_ch, w.n_s))
    a, b = 1.75, -0.6
    _close(D.das_workload(a * r1 + b * r2, w),
           a * D.das_workload(r1, w) + b * D.das_workload(r2, w), rtol=1e-12, atol=1e-12,
           msg="linearity")


def pin_mirror_symmetry():
    """Mirror-symmetric phantom and symmetric angle set -> y(x) = y(-x)."""
    w = phantom.tiny_pwi(n_elem=16, n_ch=16, n_tx=4, angles_deg=(-12.0, -3.0, 3.0, 12.0),
                         n_s=1024, nz=21, nx=15, z_min=6e-3, z_max=9e-3,
                         x_min=-2.1e-3, x_max=2.1e-3)
    rf = (phantom.point_echo_rf(w, 1.1e-3, 7.3e-3) + phantom.point_echo_rf(w, -1.1e-3, 7.3e-3)
          + 0.5 * phantom.point_echo_rf(w, 0.4e-3, 8.2e-3)
          + 0.5 * phantom.point_echo_rf(w, -0.4e-3, 8.2e-3))
    y = D.das_workload(rf, w)
    _close(y, y[:, ::-1], rtol=1e-9, atol=1e-9 * np.abs(y).max(), msg="mirror symmetry")


def pin_stai_reciprocity():
    """STAI with transmit set = receive set: swapping the transmit and
    receive roles of the RF (rf[t][j] -> rf[j][t]) leaves y unchanged."""
    w = phantom.tiny_stai(f_number=0.0)
    rng = np.random.default_rng(6)
    rf = rng.normal(size=(w.n_tx, w.n_ch, w.n_s))
    _close(D.das_workload(rf, w), D.das_workload(rf.transpose(1, 0, 2), w), rtol=1e-12,
           atol=1e-12, msg="reciprocity")


def _brute(rf, w):
    """Pure-Python scalar loops, written from the definitions."""
    g = w.grid()
    ex = [(e - (w.n_elem - 1) / 2) * w.pitch for e in range(w.n_elem)]
    out = np.zeros((w.nz, w.nx))
    for iz in range(w.nz):
        z = g["z0"] + iz * g["dz"]
        for ix in range(w.nx):
            x = g["x0"] + ix * g["dx"]
            acc = 0.0
            for t in range(w.n_tx):
                if w.mode == "stai":
                    e = w.tx_elements()[t]
                    ttx = math.sqrt((x - ex[e]) ** 2 + z * z) / w.c
                else:
                    th = w.angles_rad()[t]
                    off = max(-xe * math.sin(th) for xe in ex)
                    ttx = (z * math.cos(th) + x * math.sin(th) + off) / w.c
                for j in range(w.n_ch):
                    xr = ex[w.rx_elements()[j]]
                    if w.f_number > 0 and 2 * w.f_number * abs(x - xr) > z:
                        continue
                    trx = math.sqrt((x - xr) ** 2 + z * z) / w.c
                    u = (ttx + trx - w.t0) * w.fs
                    n = math.floor(u)
                    if n < 0 or n > w.n_s - 2:
                        continue
                    al = u - n
                    acc += (1 - al) * rf[t, j, n] + al * rf[t, j, n + 1]
            out[iz, ix] = acc
    return out


def pin_brute_force_tiny():
    for w in (phantom.tiny_stai(), phantom.tiny_stai(f_number=0.8, t0=0.3e-6),
              phantom.tiny_pwi(), phantom.tiny_pwi(f_number=1.2, t0=-0.2e-6)):
        rf = phantom.synth_rf(w, quantize=False)[0]
        _close(D.das_workload(rf, w), _brute(rf, w), rtol=1e-12, atol=1e-9,
               msg=f"brute force {w.name}")


# --------------------------------------------------------------------------
# envelope (analytic signal + absolute value, Fig. 2)
# --------------------------------------------------------------------------

def pin_envelope_cosine():
    for n in (64, 128, 250):
        s = np.arange(n)
        for k in (1, 5, n // 2 - 1):
            y = np.cos(2 * np.pi * k * s / n + 0.3)
            a = E.analytic_signal(y[:, None])[:, 0]
            _close(np.abs(a), np.ones(n), atol=1e-12, rtol=0, msg=f"|analytic(cos)| n={n} k={k}")
            # the analytic signal of cos is cos + i sin
            _close(a.imag, np.sin(2 * np.pi * k * s / n + 0.3), atol=1e-12, rtol=0,
                   msg="quadrature of cos is sin")


def pin_envelope_gaussian():
    """Gaussian-modulated cosine with the generator's pulse width: envelope is
    the Gaussian (product theorem; spectral overlap below 1e-6)."""
    fs, fc = 50e6, 5e6
    sig = 2.0 / (fc * 2.0 * math.sqrt(2.0 * math.log(2.0))) * fs  # samples
    n = 512
    s = np.arange(n)
    g = np.exp(-((s - 200.3) ** 2) / (2 * sig * sig))
    y = g * np.cos(2 * np.pi * fc / fs * (s - 200.3) + 0.4)
    env = E.envelope(y[:, None])[:, 0]
    _close(env, g, atol=1e-6, rtol=0, msg="Gaussian envelope")


def pin_envelope_constant_and_scipy():
    y = np.full((32, 3), -2.5)
    _close(E.envelope(y), np.full((32, 3), 2.5), atol=1e-12, rtol=0, msg="DC")
    import scipy.signal

    rng = np.random.default_rng(8)
    for n in (64, 65, 100):
        y = rng.normal(size=(n, 4))
        _close(E.analytic_signal(y), scipy.signal.hilbert(y, axis=0), atol=1e-12, rtol=0,
               msg=f"scipy hilbert n={n}")


# --------------------------------------------------------------------------
# log compression / clip
# --------------------------------------------------------------------------

def pin_bmode_golden():
    g = json.load(open(os.path.join(GOLDEN, "bmode_closed_form.json")))
    m, dr = g["frame_max"], g["dr_db"]
    env = [m * 10 ** (c["env_over_max_db"] / 20) if not c.get("env_zero") else 0.0
           for c in g["cases"]]
    exp = [c["expected_db"] for c in g["cases"]]
    env = np.array(env)[:, None]
    _close(B.log_compress(env, dr), np.array(exp)[:, None], atol=1e-10, rtol=0, msg="dB golden")
    _close(B.log_compress(env, dr, offset=True), np.array(exp)[:, None] + dr, atol=1e-10,
           rtol=0, msg="dB offset")


def pin_bmode_per_frame_and_degenerate():
    rng = np.random.default_rng(9)
    e = np.abs(rng.normal(size=(2, 8, 8)))
    e[1] *= 1000.0
    b = B.log_compress(e, 40.0)
    for f in range(2):
        assert b[f].max() == 0.0, "each frame's maximum maps to 0 dB"
        _close(b[f], np.clip(20 * np.log10(e[f] / e[f].max()), -40, 0), atol=1e-12, rtol=0,
               msg="per-frame reference")
    z = B.log_compress(np.zeros((4, 4)), 30.0)
    _close(z, np.full((4, 4), -30.0), atol=0, rtol=0, msg="all-zero frame")
    assert np.all(np.isfinite(z))


def pin_bmode_gaussian_pulses():
    """The whole frame step (Fig. 2: analytic signal -> absolute value ->
    dynamic adjustment) on a frame of depth columns whose B-mode is known in
    closed form: column k holds a_k g(z) cos(2 pi fc z / fs + phi_k) with g the
    Gaussian of the generator's pulse width, so its envelope is a_k g(z)
    (product theorem, leakage < 1e-6 of the peak) and its dB image is
    20 log10(a_k g(z) / max_k a_k) clipped to [-DR, 0] - the reference being
    the frame maximum, which lies in another column for all but one.  A zero
    column maps to -DR.  Two frames with different peak columns and scales
    check that each frame takes its own maximum."""
    fs, fc, dr = 50e6, 5e6, 60.0
    sig = 2.0 / (fc * 2.0 * math.sqrt(2.0 * math.log(2.0))) * fs  # samples
    nz = 512
    s = np.arange(nz, dtype=np.float64)
    frames = [((1.0, 0.25, 3.0, 0.0), (180.0, 300.0, 256.0, 0.0)),
              ((40.0, 0.0, 7.5, 400.0), (128.0, 0.0, 333.0, 251.0))]
    y = np.zeros((len(frames), nz, 4))
    exp = np.zeros_like(y)
    for f, (amps, centres) in enumerate(frames):
        top = max(amps)
        for k, (a, c) in enumerate(zip(amps, centres)):
            g = np.exp(-((s - c) ** 2) / (2 * sig * sig))
            y[f, :, k] = a * g * np.cos(2 * np.pi * fc / fs * (s - c) + 0.7 * k + 0.2)
            with np.errstate(divide="ignore"):
                exp[f, :, k] = np.clip(20 * np.log10(a * g / top), -dr, 0.0)
    got = B.bmode(y, dr)
    for f in range(len(frames)):
        # the envelope is a g to ~1e-6 of the column peak: compare where the
        # expected level is above -40 dB of the frame (<= 3e-3 dB there), and
        # require the clip floor well below it
        on = exp[f] > -40.0
        _close(got[f][on], exp[f][on], atol=3e-3, rtol=0, msg=f"bmode frame {f}")
        deep = exp[f] <= -dr
        assert np.all(got[f][deep & (exp[f] <= -dr)] >= -dr)
        far = np.zeros_like(deep)
        for k, (a, c) in enumerate(zip(*frames[f])):
            far[:, k] = np.abs(s - c) > 8 * sig if a > 0 else True
        assert np.all(got[f][far] == -dr), f"frame {f}: far from every pulse is clipped"
        assert got[f].max() == 0.0 or abs(got[f].max()) < 1e-5, "frame maximum maps to 0 dB"
    offs = B.bmode(y, dr, offset=True)
    _close(offs, got + dr, atol=1e-12, rtol=0, msg="bmode offset")


# --------------------------------------------------------------------------
# derivatives (adjoint w.r.t. RF, derivative w.r.t. the speed of sound)
# --------------------------------------------------------------------------

def pin_adjoint_dot_product():
    """<A r, g> = <r, A^T g> for the (pinned) forward A."""
    rng = np.random.default_rng(21)
    for w in (phantom.tiny_stai(f_number=0.8, t0=0.3e-6), phantom.tiny_pwi(f_number=1.2)):
        r = rng.normal(size=(w.n_tx, w.n_ch, w.n_s))
        g = rng.normal(size=(w.nz, w.nx))
        lhs = float(np.sum(D.das_workload(r, w) * g))
        rhs = float(np.sum(r * A.das_adjoint_workload(g, w)))
        _close(lhs, rhs, rtol=1e-12, atol=1e-12, msg=f"adjoint dot product {w.name}")


def pin_dydc_linear_ramp():
    """r[s] = a + b s: y = sum (a + b u) exactly, so dy/dc = b sum du/dc with
    du/dc = -(tau_tx + tau_rx) fs / c (times of flight are lengths over c)."""
    a, b = 2.0, -0.375
    for w in (_deep_stai(), phantom.tiny_pwi(n_elem=8, n_ch=8, n_s=4096, nz=5, nx=7,
                                             z_min=4e-3, z_max=12e-3)):
        rf = np.broadcast_to(a + b * np.arange(w.n_s, dtype=np.float64),
                             (w.n_tx, w.n_ch, w.n_s))
        got = A.das_dydc_workload(rf, w)
        ttx, trx = D.workload_tof(w)
        exp = b * sum(-(ttx[t][None] + trx).sum(axis=0) * w.fs / w.c for t in range(w.n_tx))
        _close(got, exp, rtol=1e-10, msg=f"dy/dc ramp {w.name}")
        # and the same against a central difference of the forward (linear in u)
        h = 1e-3
        fd = (D.das_workload(rf, w.with_(c=w.c + h)) - D.das_workload(rf, w.with_(c=w.c - h))) / (2 * h)
        _close(got, fd, rtol=1e-6, msg=f"dy/dc ramp vs central difference {w.name}")


# --------------------------------------------------------------------------
# FIR pre-filter (Sec. II-B pre-processing op)
# --------------------------------------------------------------------------

def pin_fir_impulse_and_numpy():
    rng = np.random.default_rng(31)
    for k_len in (1, 7, 31):
        h = rng.normal(size=k_len)  # no symmetry: a reversed filter fails
        d = (k_len - 1) // 2
        x = np.zeros(96)
        x[40] = 1.0
        y = F.fir_same(x, h)
        # an impulse at s0 returns the taps at s0 - D ... s0 + D, zeros elsewhere
        exp = np.zeros(96)
        exp[40 - d:40 + d + 1] = h
        _close(y, exp, rtol=0, atol=1e-15, msg=f"fir impulse K={k_len}")
        # the definition is numpy's centred convolution, rows filtered separately
        r = rng.normal(size=(3, 2, 64))
        got = F.fir_same(r, h)
        ref = np.stack([[np.convolve(r[a, b], h, mode="same") for b in range(2)]
                        for a in range(3)])
        _close(got, ref, rtol=1e-12, atol=1e-12, msg=f"fir vs numpy.convolve K={k_len}")


def pin_fir_moving_average_tone():
    # K-tap moving average of a tone: gain sin(pi f K / fs) / (K sin(pi f / fs))
    # (Dirichlet kernel), zero phase for the centred filter, away from edges
    k_len, fs, f0, s_len = 9, 50e6, 3.1e6, 400
    h = np.full(k_len, 1.0 / k_len)
    s = np.arange(s_len)
    x = np.cos(2 * np.pi * f0 * s / fs + 0.4)
    gain = math.sin(math.pi * f0 * k_len / fs) / (k_len * math.sin(math.pi * f0 / fs))
    y = F.fir_same(x, h)
    d = (k_len - 1) // 2
    _close(y[d:s_len - d], gain * x[d:s_len - d], rtol=0, atol=1e-12, msg="fir tone gain")


def pin_fir_edges_constant():
    # r = 1: y[s] is the sum of the taps that land inside the record; with
    # h[k] = k + 1 the partial sums are arithmetic series
    k_len, s_len = 11, 40
    d = (k_len - 1) // 2
    h = np.arange(1, k_len + 1, dtype=np.float64)
    y = F.fir_same(np.ones(s_len), h)
    total = k_len * (k_len + 1) / 2
    for s in range(s_len):
        # taps k with 0 <= s + d - k < S  <=>  s + d - S < k <= s + d
        k_hi = min(k_len - 1, s + d)
        k_lo = max(0, s + d - s_len + 1)
        exp = (k_hi + 1) * (k_hi + 2) / 2 - k_lo * (k_lo + 1) / 2
        assert abs(y[s] - exp) <= 1e-12, f"fir edge s={s}: {y[s]} vs {exp}"
    assert abs(y[s_len // 2] - total) <= 1e-12


# --------------------------------------------------------------------------
# qUS moment maps (Fig. 3: slice -> E[X], E[X^2], E[X^3])
# --------------------------------------------------------------------------

def pin_moments_constant_and_depth_ramp():
    env = np.full((2, 20, 12), 1.5)
    m = M.moment_maps(env, 5, 3, 2, 4)
    assert m.shape == (2, 3, 8, 3)
    for p in range(3):
        _close(m[:, p], np.full((2, 8, 3), 1.5 ** (p + 1)), rtol=1e-14, msg="moments constant")
    # env = depth index z: window rows a..a+wz-1, Faulhaber sums of z, z^2, z^3
    nz, nx, wz, wx, sz, sx = 23, 9, 6, 4, 3, 2
    env = np.broadcast_to(np.arange(nz, dtype=np.float64)[:, None], (nz, nx)).copy()
    m = M.moment_maps(env, wz, wx, sz, sx)
    mz, mx = (nz - wz) // sz + 1, (nx - wx) // sx + 1
    assert m.shape == (3, mz, mx)

    def s_pow(n, p):  # sum_{z=0}^{n-1} z^p
        return [n, n * (n - 1) / 2, (n - 1) * n * (2 * n - 1) / 6, ((n - 1) * n / 2) ** 2][p]

    for i in range(mz):
        a = i * sz
        for p in (1, 2, 3):
            exp = (s_pow(a + wz, p) - s_pow(a, p)) / wz
            _close(m[p - 1, i], np.full(mx, exp), rtol=1e-13, msg=f"moments ramp p={p} i={i}")


def pin_moments_lateral_index_and_brute():
    rng = np.random.default_rng(32)
    # env = lateral index x: E[X] of window j is j sx + (wx - 1) / 2
    env = np.broadcast_to(np.arange(17, dtype=np.float64)[None, :], (8, 17)).copy()
    m = M.moment_maps(env, 3, 5, 1, 3)
    exp = np.arange(m.shape[2]) * 3 + 2.0
    _close(m[0], np.broadcast_to(exp, m[0].shape), rtol=1e-14, msg="moments lateral placement")
    # brute force, scalar loops
    env = rng.rayleigh(1.0, size=(2, 11, 10))
    wz, wx, sz, sx = 4, 3, 3, 2
    got = M.moment_maps(env, wz, wx, sz, sx)
    for f in range(2):
        for i in range((11 - wz) // sz + 1):
            for j in range((10 - wx) // sx + 1):
                vals = [env[f, i * sz + a, j * sx + b] for a in range(wz) for b in range(wx)]
                for p in (1, 2, 3):
                    exp = sum(v ** p for v in vals) / len(vals)
                    assert abs(got[f, p - 1, i, j] - exp) <= 1e-12 * max(1.0, exp)


def pin_moments_rayleigh():
    # envelope of circular complex Gaussian speckle: Rayleigh(sigma) with
    # E[X] = sigma sqrt(pi/2), E[X^2] = 2 sigma^2, E[X^3] = 3 sigma^3 sqrt(pi/2)
    rng = np.random.default_rng(33)
    sigma = 0.7
    z = rng.normal(0, sigma, size=(512, 512)) + 1j * rng.normal(0, sigma, size=(512, 512))
    m = M.moment_maps(np.abs(z), 256, 256, 256, 256)
    exp = (sigma * math.sqrt(math.pi / 2), 2 * sigma ** 2, 3 * sigma ** 3 * math.sqrt(math.pi / 2))
    for p in range(3):
        _close(m[p], np.full((2, 2), exp[p]), rtol=0.02, msg=f"Rayleigh moment {p + 1}")


ALL_PINS = [
    pin_tof_golden,
    pin_pwi_wavefront_geometry,
    pin_constant_rf_counts,
    pin_linear_ramp,
    pin_window_edges,
    pin_point_scatterer_focus,
    pin_linearity,
    pin_mirror_symmetry,
    pin_stai_reciprocity,
    pin_brute_force_tiny,
    pin_envelope_cosine,
    pin_envelope_gaussian,
    pin_envelope_constant_and_scipy,
    pin_bmode_golden,
    pin_bmode_per_frame_and_degenerate,
    pin_bmode_gaussian_pulses,
    pin_adjoint_dot_product,
    pin_dydc_linear_ramp,
    pin_fir_impulse_and_numpy,
    pin_fir_moving_average_tone,
    pin_fir_edges_constant,
    pin_moments_constant_and_depth_ramp,
    pin_moments_lateral_index_and_brute,
    pin_moments_rayleigh,
]
