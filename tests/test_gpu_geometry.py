"""DAS geometry coverage on the GPU, through the C ABI, against the FP64
oracle: the served mixed-stream shape classes (array sizes 64/128/192,
transmit counts 16-128 with STAI transmit subsets, records 1024-4096,
grids 256 x 128 to 1024 x 512 - each picks its own launch shape), and an
array with explicit, non-uniform element positions.

Bar: normalised L2 <= 1e-5 (FP32 compute; the oracle is fed the very RF
values the kernel reads).  The served classes are checked on whole sampled
columns of the full grid, computed in the launch the server uses.
"""

import dataclasses

import numpy as np
import pytest

import oracle
import phantom
from oracle.das import workload_pixels
from phantom.configs import served_mix
from wfhelp import nl2, scan_from_workload

pytestmark = pytest.mark.gpu

NL2_TOL = 1e-5
# (mode, N, T, S, nz, nx): spans the launch shapes and the extremes of the mix
CLASSES = [
    ("stai", 64, 16, 1024, 256, 128),
    ("stai", 64, 64, 4096, 512, 256),
    ("stai", 192, 128, 2048, 1024, 512),
    ("stai", 128, 32, 1024, 1024, 512),
    ("pwi", 64, 16, 4096, 1024, 512),
    ("pwi", 192, 128, 1024, 256, 128),
    ("pwi", 128, 64, 2048, 512, 256),
    ("pwi", 192, 32, 4096, 256, 128),
]


def _class(mode, n, t, s, nz, nx):
    for w in served_mix():
        if (w.mode, w.n_elem, w.n_tx, w.n_s, w.nz, w.nx) == (mode, n, t, s, nz, nx):
            rng = np.random.default_rng(n * 1000 + t)
            xs = w.elem_x()
            pts = dict(x=tuple(rng.uniform(xs[0], xs[-1], 12)),
                       z=tuple(rng.uniform(6e-3, 29e-3, 12)))
            return w.with_(phantom="points", phantom_args=pts)
    raise KeyError((mode, n, t, s, nz, nx))


@pytest.mark.parametrize("cls", CLASSES, ids=lambda c: "_".join(map(str, c)))
def test_served_class_sampled_columns(wf_gpu, cls):
    import torch

    w = _class(*cls)
    rf = phantom.synth_rf(w)[0]
    y = wf_gpu.das(scan_from_workload(w), torch.from_numpy(rf).cuda())
    torch.cuda.synchronize()
    cols = sorted({0, w.nx // 3, w.nx - 1})
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(np.asarray(cols), (w.nz, 1))
    ref = oracle.das_workload(rf.astype(np.float64), w, iz, ix)
    err = nl2(y.cpu().numpy()[:, cols], ref)
    info = wf_gpu.tile_info(scan_from_workload(w), w.n_s)
    print(f"{w.name}: nL2 {err:.2e} (tile {info['threads']} x {info['px']}, "
          f"{info['tile_z']} x {info['tile_x']})")
    assert err <= NL2_TOL


@pytest.mark.parametrize("mode", ["stai", "pwi"])
def test_jittered_element_positions(wf_gpu, mode):
    """Element positions passed explicitly (uniform pitch plus up to 30 %
    jitter); the oracle uses the same positions."""
    import torch

    base = phantom.tiny_stai(n_s=128) if mode == "stai" else phantom.tiny_pwi(n_s=128)
    w = base.with_(nz=24, nx=20, z_min=0.5e-3, z_max=2.5e-3, f_number=0.6)
    rng = np.random.default_rng(21)
    ex = np.asarray(w.elem_x()) + rng.uniform(-0.3, 0.3, w.n_elem) * w.pitch
    scan = dataclasses.replace(scan_from_workload(w), elem_x=tuple(float(v) for v in ex))
    rf = rng.normal(size=(w.n_tx, w.n_ch, w.n_s)).astype(np.float32)
    y = wf_gpu.das(scan, torch.from_numpy(rf).cuda()[None])
    torch.cuda.synchronize()
    x, z = workload_pixels(w)
    common = dict(c=w.c, fs=w.fs, t0=w.t0, f_number=w.f_number)
    if mode == "stai":
        ref = oracle.das_stai(rf.astype(np.float64), x, z, ex, w.tx_elements(), w.rx_elements(),
                              **common)
    else:
        ref = oracle.das_pwi(rf.astype(np.float64), x, z, ex, w.angles_rad(), w.rx_elements(),
                             tref=w.tref, **common)
    err = nl2(y[0].cpu().numpy(), ref)
    print(f"jittered {mode}: nL2 {err:.2e}")
    assert err <= NL2_TOL
