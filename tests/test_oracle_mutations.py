"""Plant plausible mistakes in the oracle (on the CPU) and check that at least
one pin catches each: the pins are only worth something if they fail on a
dropped term, a wrong sign or index, or a transposed operand."""

import math

import numpy as np
import pytest

import oracle_pins as P
from oracle import adjoint as A
from oracle import analytic as E
from oracle import das as D
from oracle import dbclip as B
from oracle import fir as F
from oracle import moments as M

_orig_interp = D.interp_linear
_orig_tof_rx = D.tof_receive
_orig_pixels = D.pixel_positions
_orig_logc = B.log_compress


def _interp_floor_only(row, u):
    u = np.asarray(u, dtype=np.float64)
    n = np.floor(u)
    ok = (n >= 0) & (n <= row.shape[0] - 2)
    return np.where(ok, row[np.where(ok, n, 0).astype(np.int64)], 0.0)


def _interp_swapped_weights(row, u):
    u = np.asarray(u, dtype=np.float64)
    n = np.floor(u)
    a = u - n
    ok = (n >= 0) & (n <= row.shape[0] - 2)
    ni = np.where(ok, n, 0).astype(np.int64)
    return np.where(ok, a * row[ni] + (1 - a) * row[np.minimum(ni + 1, row.shape[0] - 1)], 0.0)


def _interp_window_to_last(row, u):
    # accepts n = S-1 (reads past the pair) instead of stopping at S-2
    u = np.asarray(u, dtype=np.float64)
    s = row.shape[0]
    n = np.floor(u)
    a = u - n
    ok = (n >= 0) & (n <= s - 1)
    ni = np.where(ok, n, 0).astype(np.int64)
    return np.where(ok, (1 - a) * row[ni] + a * row[np.minimum(ni + 1, s - 1)], 0.0)


def _tof_pwi_sign(x, z, theta, elem_x, c, tref="first"):
    o = D.pwi_time_offset(theta, elem_x, tref)
    return (np.asarray(z) * math.cos(theta) - np.asarray(x) * math.sin(theta) + o) / c


def _tof_rx_no_depth(x, z, x_elem, c):
    return np.abs(np.asarray(x) - x_elem) / c + 0.0 * np.asarray(z)


def _frac_t0_sign(tau_tx, tau_rx, t0, fs):
    return (np.asarray(tau_tx) + np.asarray(tau_rx) + t0) * fs


def _frac_no_tx(tau_tx, tau_rx, t0, fs):
    return (2 * np.asarray(tau_rx) - t0) * fs


def _weight_no_factor2(x, z, x_elem, f_number):
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if f_number <= 0:
        return np.ones(np.broadcast(x, z).shape)
    return (f_number * np.abs(x - x_elem) <= z).astype(np.float64)


def _pixels_transposed(nz, nx, z0, dz, x0, dx):
    x, z = _orig_pixels(nz, nx, z0, dz, x0, dx)
    iz = np.arange(nz, dtype=np.float64)[:, None]
    ix = np.arange(nx, dtype=np.float64)[None, :]
    # lateral index drives x through dz's step and vice versa
    return np.broadcast_to(x0 + iz * dx, (nz, nx)).copy(), np.broadcast_to(z0 + ix * dz, (nz, nx)).copy()


def _h_no_doubling(n):
    h = np.zeros(n)
    if n:
        h[0] = 1.0
        h[1 : (n + 1) // 2] = 1.0
    return h


def _h_negative_side(n):
    h = np.zeros(n)
    if n:
        h[0] = 1.0
        h[n // 2 + 1 :] = 2.0
        if n % 2 == 0:
            h[n // 2] = 1.0
    return h


def _analytic_wrong_axis(y, axis=-2):
    y = np.asarray(y, dtype=np.float64)
    spec = np.fft.fft(y, axis=-1)
    n = y.shape[-1]
    return np.fft.ifft(spec * E.hilbert_multiplier(n), axis=-1)


def _logc_power_db(env, dr_db, offset=False):
    return _orig_logc(np.asarray(env) ** 0.5, dr_db, offset)


def _logc_global_max(env, dr_db, offset=False):
    env = np.asarray(env, dtype=np.float64)
    m = env.max()
    with np.errstate(divide="ignore"):
        b = np.where(env > 0, 20 * np.log10(env / m), -dr_db)
    b = np.clip(b, -dr_db, 0.0)
    return b + dr_db if offset else b


def _logc_no_clip(env, dr_db, offset=False):
    env = np.asarray(env, dtype=np.float64)
    e = env[None] if env.ndim == 2 else env
    out = np.stack([np.where(f > 0, 20 * np.log10(np.where(f > 0, f, 1) / f.max()), -dr_db)
                    for f in e])
    out = out[0] if env.ndim == 2 else out
    return out + dr_db if offset else out


def _adjoint_no_alpha(g, tau_tx, tau_rx, weight, t0, fs, n_s):
    # spreads (1 - a) to both samples
    g = np.asarray(g, dtype=np.float64).ravel()
    T, C = tau_tx.shape[0], tau_rx.shape[0]
    out = np.zeros((T, C, n_s))
    for t in range(T):
        for j in range(C):
            u = D.fractional_index(tau_tx[t].ravel(), tau_rx[j].ravel(), t0, fs)
            n = np.floor(u)
            a = u - n
            ok = (n >= 0) & (n <= n_s - 2)
            ni = n[ok].astype(np.int64)
            wg = (weight[j].ravel() * g)[ok]
            np.add.at(out[t, j], ni, (1.0 - a[ok]) * wg)
            np.add.at(out[t, j], ni + 1, (1.0 - a[ok]) * wg)
    return out


def _dydc_sign(rf, tau_tx, tau_rx, weight, t0, fs, c):
    return -_orig_dydc(rf, tau_tx, tau_rx, weight, t0, fs, c)


def _dydc_rx_only(rf, tau_tx, tau_rx, weight, t0, fs, c):
    return _orig_dydc(rf, np.zeros_like(tau_tx), tau_rx, weight, t0, fs, c) * 0 + \
        _orig_dydc(rf, tau_tx * 0.0 + tau_tx, tau_rx * 0.0, weight, t0, fs, c)


_orig_dydc = A.das_dydc_sum


def _bmode_no_envelope(y, dr_db, offset=False):
    # log-compresses the rectified RF instead of its envelope
    return B.log_compress(np.abs(np.asarray(y, dtype=np.float64)), dr_db, offset)


def _bmode_lateral_axis(y, dr_db, offset=False):
    # takes the analytic signal across columns instead of down each column
    return B.log_compress(E.envelope(y, axis=-1), dr_db, offset)


def _bmode_no_abs(y, dr_db, offset=False):
    # keeps the real part of the analytic signal (the RF itself)
    return B.log_compress(np.maximum(E.analytic_signal(y).real, 0.0), dr_db, offset)


_orig_fir = F.fir_same
_orig_moments = M.moment_maps


def _fir_correlation(rf, taps):
    # correlates instead of convolving (reversed taps)
    return _orig_fir(rf, np.asarray(taps, dtype=np.float64)[::-1])


def _fir_shift_one(rf, taps):
    y = _orig_fir(rf, taps)
    out = np.zeros_like(y)
    out[..., 1:] = y[..., :-1]
    return out


def _fir_circular(rf, taps):
    # wraps around the record instead of zero padding
    h = np.asarray(taps, dtype=np.float64)
    r = np.asarray(rf, dtype=np.float64)
    d = (h.shape[0] - 1) // 2
    return sum(h[k] * np.roll(r, k - d, axis=-1) for k in range(h.shape[0]))


def _fir_last_tap_dropped(rf, taps):
    h = np.array(taps, dtype=np.float64)
    h[-1] = 0.0
    return _orig_fir(rf, h)


def _moments_cube_of_mean(env, wz, wx, sz, sx):
    m = _orig_moments(env, wz, wx, sz, sx)
    m[..., 2, :, :] = m[..., 0, :, :] ** 3
    return m


def _moments_short_window(env, wz, wx, sz, sx):
    # averages one row fewer than the window
    e = np.asarray(env, dtype=np.float64)
    m = _orig_moments(e, max(1, wz - 1), wx, sz, sx)
    mz = (e.shape[-2] - wz) // sz + 1
    return m[..., :mz, :]


def _moments_swapped_window(env, wz, wx, sz, sx):
    e = np.asarray(env, dtype=np.float64)
    return np.swapaxes(_orig_moments(np.swapaxes(e, -1, -2), wz, wx, sz, sx), -1, -2)


def _moments_unit_stride(env, wz, wx, sz, sx):
    return _orig_moments(env, wz, wx, 1, 1)


MUTATIONS = {
    "interp_floor_only": (D, "interp_linear", _interp_floor_only),
    "interp_swapped_weights": (D, "interp_linear", _interp_swapped_weights),
    "interp_window_to_last": (D, "interp_linear", _interp_window_to_last),
    "pwi_offset_dropped": (D, "pwi_time_offset", lambda th, ex, tref: 0.0),
    "pwi_sin_sign": (D, "tof_pwi_transmit", _tof_pwi_sign),
    "rx_depth_dropped": (D, "tof_receive", _tof_rx_no_depth),
    "t0_sign": (D, "fractional_index", _frac_t0_sign),
    "tx_term_dropped": (D, "fractional_index", _frac_no_tx),
    "aperture_factor2_dropped": (D, "receive_weight", _weight_no_factor2),
    "grid_transposed": (D, "pixel_positions", _pixels_transposed),
    "hilbert_no_doubling": (E, "hilbert_multiplier", _h_no_doubling),
    "hilbert_negative_side": (E, "hilbert_multiplier", _h_negative_side),
    "hilbert_wrong_axis": (E, "analytic_signal", _analytic_wrong_axis),
    "db_power_not_amplitude": (B, "log_compress", _logc_power_db),
    "db_global_max": (B, "log_compress", _logc_global_max),
    "db_no_clip": (B, "log_compress", _logc_no_clip),
    "bmode_envelope_skipped": (B, "bmode", _bmode_no_envelope),
    "bmode_envelope_along_x": (B, "bmode", _bmode_lateral_axis),
    "bmode_modulus_dropped": (B, "bmode", _bmode_no_abs),
    "adjoint_weight_not_alpha": (A, "das_adjoint_sum", _adjoint_no_alpha),
    "dydc_sign": (A, "das_dydc_sum", _dydc_sign),
    "fir_correlation_not_convolution": (F, "fir_same", _fir_correlation),
    "fir_output_shifted": (F, "fir_same", _fir_shift_one),
    "fir_circular_edges": (F, "fir_same", _fir_circular),
    "fir_last_tap_dropped": (F, "fir_same", _fir_last_tap_dropped),
    "moments_cube_of_mean": (M, "moment_maps", _moments_cube_of_mean),
    "moments_short_window": (M, "moment_maps", _moments_short_window),
    "moments_window_transposed": (M, "moment_maps", _moments_swapped_window),
    "moments_stride_ignored": (M, "moment_maps", _moments_unit_stride),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    mod, attr, fn = MUTATIONS[name]
    monkeypatch.setattr(mod, attr, fn)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin()
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            caught.append(f"{pin.__name__}: {type(e).__name__}")
    assert caught, f"mutation {name} survived every pin"
