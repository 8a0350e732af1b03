"""Seeded input generator: determinism, quantisation, noise level, and that a
point echo sits at its analytic arrival time (CPU)."""

import math

import numpy as np

import phantom
from phantom import synth


def test_seeded_and_int16_full_scale():
    w = phantom.get_workload("stai_small")
    a = phantom.synth_rf(w, cache=False, workers=1)
    b = phantom.synth_rf(w, cache=False, workers=1)
    assert a.dtype == np.int16 and a.shape == (1, 32, 32, 1024)
    assert np.array_equal(a, b)
    assert int(np.abs(a).max()) == 8191


def test_noise_level_20db():
    w = phantom.get_workload("stai_small")
    clean = synth._frame_float(w, 0, 1)
    noisy = phantom.synth_rf(w.with_(snr_db=20.0), quantize=False, cache=False, workers=1)[0]
    # the record is rescaled after adding noise: remove the scaled clean part
    # (least squares) and compare RMS levels
    k = float(np.sum(noisy * clean) / np.sum(clean * clean))
    resid = noisy - k * clean
    snr = 20 * math.log10(k * math.sqrt(np.mean(clean ** 2)) / math.sqrt(np.mean(resid ** 2)))
    assert abs(snr - 20.0) < 0.3, snr


def test_point_echo_arrival_time():
    w = phantom.tiny_pwi(n_elem=8, n_ch=8, n_tx=2, angles_deg=(-9.0, 14.0), n_s=2048,
                         fs=200e6)
    x, z = 0.4e-3, 6.0e-3
    rf = phantom.point_echo_rf(w, x, z)
    ex = [(e - 3.5) * w.pitch for e in range(8)]
    for t, th in enumerate(w.angles_rad()):
        for j in range(8):
            xf = ex[0] if th > 0 else ex[-1]
            tau = ((x - xf) * math.sin(th) + z * math.cos(th) + math.hypot(x - ex[j], z)) / w.c
            env = np.abs(np.fft.ifft(np.fft.fft(rf[t, j]) * np.r_[1, 2 * np.ones(1023), 1, np.zeros(1023)]))
            peak = np.argmax(env)
            # quadratic refinement of the envelope peak
            a, b, c = env[peak - 1], env[peak], env[peak + 1]
            frac = 0.5 * (a - c) / (a - 2 * b + c)
            assert abs((peak + frac) / w.fs - tau) < 0.05 / w.fs


def test_histogram_synthesis_matches_exact():
    w = phantom.get_workload("pwi").with_(n_tx=2, angles_deg=(-16.0, 7.0), n_ch=16)
    rng = np.random.default_rng(0)
    xs = rng.uniform(-0.019, 0.019, 40)
    zs = rng.uniform(0.005, 0.03, 40)
    a = rng.normal(size=40) + 1j * rng.normal(size=40)
    for t in range(2):
        e = synth._exact_tx(w, xs, zs, a, t)
        h = synth._hist_tx(w, xs, zs, a, t)
        assert np.linalg.norm(e - h) / np.linalg.norm(e) < 5e-3


def test_cyst_interiors_are_empty():
    w = phantom.get_workload("pwi").with_(phantom_args=dict(
        n_speckle=20000, z_range_mm=(5.0, 30.0), cyst_radius_mm=2.0,
        cysts_mm=((-10.0, 12.0), (0.0, 18.0), (10.0, 24.0))))
    xs, zs, a = phantom.scatterers_for(w, 0)
    for cx, cz in ((-10.0, 12.0), (0.0, 18.0), (10.0, 24.0)):
        assert np.all(np.hypot(xs - cx * 1e-3, zs - cz * 1e-3) > 2e-3)
    assert 0.9 * 20000 < xs.size < 20000
