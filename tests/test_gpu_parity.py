"""HIP path vs the FP64 oracle, through the C ABI, on an MI355X.

Bars (the tolerances the path is held to):
  beamformed RF   normalised L2 error <= 1e-5 (FP32 compute, any RF dtype,
                  oracle fed the same RF values);
  B-mode          max |dB difference| <= 0.01 dB;
  delays          |device float-float delay - oracle| <= 1e-6 samples;
  integer-valued  bitwise (determinism, zero input).
Sizes: whole frames of small workloads and multi-tile sub-grids with ragged
edges; the full-size workloads in the launch configuration the benchmark
uses, checked on whole sampled columns the oracle computes one by one.
"""

import math

import numpy as np
import pytest

import oracle
import phantom
from phantom.configs import subgrid
from wfhelp import deep_pwi, nl2, scan_from_workload

pytestmark = pytest.mark.gpu

NL2_TOL = 1e-5
DB_TOL = 0.01


def _torch():
    import torch

    return torch


def _gpu(a, dtype=None):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _run_das(wf, w, rf_np, torch_dtype=None):
    """DAS of rf [F][T][C][S] or [T][C][S]; always returns [F][nz][nx]."""
    torch = _torch()
    rf_np = rf_np if rf_np.ndim == 4 else rf_np[None]
    rf = _gpu(rf_np, torch_dtype)
    y = wf.das(scan_from_workload(w), rf)
    torch.cuda.synchronize()
    assert y.dim() == 3
    return y.cpu().numpy().astype(np.float64)


from phantom.prepare import lighter as _lighter


SMALL = {
    "tiny_stai": lambda: phantom.tiny_stai(),
    "tiny_pwi": lambda: phantom.tiny_pwi(),
    "tiny_stai_apod_t0": lambda: phantom.tiny_stai(f_number=0.8, t0=0.3e-6),
    "tiny_pwi_apod_t0_centre": lambda: phantom.tiny_pwi(f_number=1.2, t0=-0.2e-6, tref="centre"),
    "single_pixel": lambda: phantom.tiny_pwi(nz=1, nx=1, z_min=0.5e-3, z_max=0.5e-3),
    # the longest record the API takes (32768 samples), imaged near its end
    "long_record": lambda: phantom.tiny_pwi(name="long_record", n_s=32768, nz=40, nx=7,
                                            z_min=0.4500, z_max=0.4512),
    "stai_small": lambda: phantom.get_workload("stai_small"),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_das_small_whole_frame(wf_gpu, name):
    w = SMALL[name]()
    rf = phantom.synth_rf(w)[0]
    y = _run_das(wf_gpu, w, rf)[0]
    ref = oracle.das_workload(rf.astype(np.float64), w)
    err = nl2(y, ref)
    print(f"{name}: nL2 {err:.3e}")
    assert err <= NL2_TOL


# multi-tile sub-windows of the full-size geometries with ragged edges
SUB = {
    "stai_full_sub": ("stai_full", 400, 132, 100, 38),
    "pwi_sub": ("pwi", 300, 131, 200, 51),
    "pwi_sub_edge": ("pwi", 960, 64, 470, 42),
    "paper_stai_sub": ("paper_stai", 900, 70, 40, 20),
    "paper_pwi_sub": ("paper_pwi", 200, 70, 50, 33),
}


@pytest.mark.parametrize("name", sorted(SUB))
def test_das_subgrid(wf_gpu, name):
    base, iz0, nz, ix0, nx = SUB[name]
    w = _lighter(phantom.get_workload(base))
    rf = phantom.synth_rf(w)[0]
    ws = subgrid(w, iz0, nz, ix0, nx)
    y = _run_das(wf_gpu, ws, rf)[0]
    ref = oracle.das_workload(rf.astype(np.float64), ws)
    err = nl2(y, ref)
    print(f"{name}: nL2 {err:.3e}")
    assert err <= NL2_TOL


@pytest.mark.parametrize("dtype", ["float16", "float32"])
def test_das_rf_dtypes(wf_gpu, dtype):
    torch = _torch()
    w = subgrid(_lighter(phantom.get_workload("pwi")), 500, 70, 100, 40)
    rf = phantom.synth_rf(w)[0]
    if dtype == "float16":
        vals = (rf.astype(np.float32) * 2.0 ** -13).astype(np.float16)
        tdt = torch.float16
    else:
        vals = rf.astype(np.float32) * 0.37
        tdt = torch.float32
    y = _run_das(wf_gpu, w, vals, tdt)[0]
    ref = oracle.das_workload(vals.astype(np.float64), w)
    err = nl2(y, ref)
    print(f"{dtype}: nL2 {err:.3e}")
    assert err <= NL2_TOL


# Batches run several frames per workgroup on the large tiles (groups of 4,
# the last one ragged here); every frame must equal its single-frame run.
# The extra cases draw uniform random records: the check needs no echoes.
@pytest.mark.parametrize("name,frames,z0,nz,x0,nx,rand", [
    ("pwi", 3, 200, 64, 300, 32, False),        # 1024-thread tiles, one ragged group
    ("pwi", 5, 200, 128, 300, 96, True),        # 1024-thread tiles, groups of 4 and 1
    ("stai_full", 6, 100, 128, 60, 64, True),   # 512-thread tiles, groups of 4 and 2
])
def test_das_multi_frame_matches_single(wf_gpu, name, frames, z0, nz, x0, nx, rand):
    w = subgrid(_lighter(phantom.get_workload(name)).with_(n_frames=frames), z0, nz, x0, nx)
    if rand:
        w = w.with_(phantom="random")
    rf = phantom.synth_rf(w)
    y = _run_das(wf_gpu, w, rf)
    for f in range(frames):
        y1 = _run_das(wf_gpu, w.with_(n_frames=1), rf[f])[0]
        assert np.array_equal(y[f], y1), f
    ref = oracle.das_workload(rf[frames - 1].astype(np.float64), w.with_(n_frames=1))
    assert nl2(y[frames - 1], ref) <= NL2_TOL


def test_das_deterministic_and_zero(wf_gpu):
    w = subgrid(_lighter(phantom.get_workload("stai_full")), 100, 64, 60, 48)
    rf = phantom.synth_rf(w)[0]
    a = _run_das(wf_gpu, w, rf)
    b = _run_das(wf_gpu, w, rf)
    assert np.array_equal(a, b)
    z = _run_das(wf_gpu, w, np.zeros_like(rf))
    assert np.all(z == 0.0)


@pytest.mark.parametrize("name", ["tiny_stai_apod_t0", "tiny_pwi_apod_t0_centre"])
def test_delays_match_oracle(wf_gpu, name):
    w = SMALL[name]()
    tx, rx = wf_gpu.delays(scan_from_workload(w))
    ttx, trx = oracle.workload_tof(w)
    e_tx = np.max(np.abs(tx.cpu().numpy() - (ttx - w.t0) * w.fs))
    e_rx = np.max(np.abs(rx.cpu().numpy() - trx * w.fs))
    print(f"{name}: delay err tx {e_tx:.2e} rx {e_rx:.2e} samples")
    assert e_tx <= 1e-6 and e_rx <= 1e-6


def test_delays_full_size_pwi(wf_gpu):
    w = phantom.get_workload("pwi")
    tx, rx = wf_gpu.delays(scan_from_workload(w))
    rng = np.random.default_rng(1)
    iz = rng.integers(0, w.nz, 2000)
    ix = rng.integers(0, w.nx, 2000)
    ttx, trx = oracle.workload_tof(w, iz, ix)
    e_tx = np.max(np.abs(tx.cpu().numpy()[:, iz, ix] - ttx * w.fs))
    e_rx = np.max(np.abs(rx.cpu().numpy()[:, iz, ix] - trx * w.fs))
    print(f"pwi full: delay err tx {e_tx:.2e} rx {e_rx:.2e} samples")
    assert e_tx <= 1e-6 and e_rx <= 1e-6


# ---------------------------------------------------------------------------
# envelope / log compression
# ---------------------------------------------------------------------------

# narrow frames take one column per workgroup; wide ones 2 (1024 x 513,
# 512 x 129 x 8, 1024 x 512) or 4 (256 x 2050, 1024 x 512 x 8) adjacent
# columns, with a ragged last group where nx is not a multiple
@pytest.mark.parametrize("nz,nx,frames", [(64, 5, 1), (1024, 33, 2), (4096, 3, 1), (2, 4, 1),
                                           (512, 7, 2), (2048, 5, 1), (4, 9, 1),
                                           (1024, 513, 1), (512, 129, 8), (1024, 512, 1),
                                           (256, 2050, 1), (1024, 512, 8)])
def test_envelope_matches_oracle(wf_gpu, nz, nx, frames):
    torch = _torch()
    rng = np.random.default_rng(nz + nx)
    y = rng.normal(size=(frames, nz, nx)).astype(np.float32)
    env, cm = wf_gpu.envelope(_gpu(y))
    torch.cuda.synchronize()
    ref = oracle.envelope(y.astype(np.float64))
    e = env.cpu().numpy()
    err = np.max(np.abs(e - ref)) / np.max(ref)
    print(f"envelope {nz}x{nx}x{frames}: max rel err {err:.2e}")
    assert err <= 1e-5
    assert np.allclose(cm.cpu().numpy(), e.max(axis=1), rtol=0, atol=0)


def test_log_compress_matches_oracle(wf_gpu):
    torch = _torch()
    rng = np.random.default_rng(3)
    env = np.abs(rng.normal(size=(2, 64, 40))).astype(np.float32)
    env[0, 3, 4] = 0.0
    env[1] *= 1e-3
    cm = env.max(axis=1)
    out = wf_gpu.log_compress(_gpu(env), _gpu(cm), 60.0)
    off = wf_gpu.log_compress(_gpu(env), _gpu(cm), 60.0, offset=True)
    torch.cuda.synchronize()
    ref = oracle.log_compress(env.astype(np.float64), 60.0)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-3
    assert np.max(np.abs(off.cpu().numpy() - (ref + 60.0))) <= 1e-3
    assert out.cpu().numpy()[0, 3, 4] == -60.0
    z = wf_gpu.log_compress(_gpu(np.zeros_like(env)), _gpu(np.zeros_like(cm)), 30.0)
    assert np.all(z.cpu().numpy() == -30.0)


@pytest.mark.parametrize("name", ["stai_small", "tiny_pwi"])
def test_bmode_end_to_end_small(wf_gpu, name):
    torch = _torch()
    w = SMALL[name]().with_(nz=64) if name == "tiny_pwi" else SMALL[name]()
    rf = phantom.synth_rf(w)[0]
    y = wf_gpu.das(scan_from_workload(w), _gpu(rf))
    b = wf_gpu.bmode(y, w.dr_db)
    torch.cuda.synchronize()
    ref = oracle.bmode(oracle.das_workload(rf.astype(np.float64), w), w.dr_db)
    d = np.max(np.abs(b.cpu().numpy() - ref))
    print(f"{name}: max |dB diff| {d:.2e}")
    assert d <= DB_TOL


# ---------------------------------------------------------------------------
# full-size workloads, launch configuration of the benchmark, sampled columns
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,cols", [("pwi", (0, 97, 255, 256, 511)),
                                       ("stai_full", (0, 64, 131, 255))])
def test_full_size_sampled_columns(wf_gpu, name, cols):
    torch = _torch()
    w = phantom.get_workload(name)
    rf = phantom.synth_rf(w)[0]
    y = wf_gpu.das(scan_from_workload(w), _gpu(rf))
    b = wf_gpu.bmode(y, w.dr_db)
    torch.cuda.synchronize()
    yc = y.cpu().numpy()
    bc = b.cpu().numpy()
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(np.asarray(cols), (w.nz, 1))
    ref = oracle.das_workload(rf.astype(np.float64), w, iz, ix)
    err = nl2(yc[:, list(cols)], ref)
    # envelope of whole columns; dB relative to each column's own maximum
    # (the frame maximum needs every column, so compare within columns)
    env_ref = oracle.envelope(ref)
    db_ref = 20 * np.log10(np.maximum(env_ref, 1e-30) / env_ref.max(axis=0))
    bsel = bc[:, list(cols)]
    db_gpu = bsel - bsel.max(axis=0)
    # the frame-level clip floor -DR, seen relative to each column maximum
    floor = -w.dr_db - bsel.max(axis=0)
    mask = db_ref > (floor + 1.0)  # clear of the clip floor
    d = np.max(np.abs(db_gpu[mask] - db_ref[mask]))
    print(f"{name} full: nL2 {err:.3e}, max |dB diff| within columns {d:.2e}")
    assert err <= NL2_TOL
    assert d <= DB_TOL
    assert bc.max() == 0.0 and bc.min() >= -w.dr_db


@pytest.mark.parametrize("name", ["stai_small", "paper_pwi", "stai_full"])
def test_das_channel_split_matches_unsplit(wf_gpu, name):
    """Grids with uneven or too little work per tile share each tile's
    channels (and transmits) among several workgroups, launched from a
    heaviest-first work list (partial frames summed in split order); without
    a workspace the same call runs unsplit.  Both agree with the oracle and
    with each other to FP32 rounding, and each is bitwise repeatable."""
    torch = _torch()
    w = phantom.get_workload(name)
    scan = scan_from_workload(w)
    need = wf_gpu.das_workspace_bytes(scan, w.n_s, 1)
    assert need > 0  # the geometry splits
    rf = _gpu(phantom.synth_rf(w))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    split = wf_gpu.das(scan, rf, workspace=ws)
    split2 = wf_gpu.das(scan, rf, workspace=ws)
    plain = wf_gpu.das(scan, rf, workspace=torch.empty(0, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(split, split2)
    cols = (0, w.nx // 2, w.nx - 1)
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(np.asarray(cols), (w.nz, 1))
    ref = oracle.das_workload(phantom.synth_rf(w)[0].astype(np.float64), w, iz, ix)
    err = nl2(split[0].cpu().numpy()[:, list(cols)], ref)
    err_plain = nl2(plain[0].cpu().numpy()[:, list(cols)], ref)
    mutual = nl2(split.cpu().numpy(), plain.cpu().numpy())
    print(f"{name} split: nL2 {err:.2e}, unsplit {err_plain:.2e}, split vs unsplit {mutual:.2e}")
    assert err <= NL2_TOL and err_plain <= NL2_TOL
    # the same FP32 terms summed in two orders (up to 16384 per pixel on the
    # full STAI frame, with heavy cancellation): each is held to the parity
    # bar, so their difference is too
    assert mutual <= NL2_TOL


def test_das_record_limited_grid(wf_gpu):
    """A grid reaching deeper than the record: tiles no window of which
    reaches into the record are left out of the work list and their pixels
    are cleared.  With and without a workspace the frame matches the
    oracle, and rows that no echo inside the record reaches are exactly 0."""
    torch = _torch()
    w = deep_pwi()
    scan = scan_from_workload(w)
    info = wf_gpu.tile_info(scan, w.n_s)
    assert info["workgroups"] < info["ntz"] * info["ntx"] * info["nsplit"]
    rf_np = phantom.synth_rf(w)
    rf = _gpu(rf_np)
    need = wf_gpu.das_workspace_bytes(scan, w.n_s, 1)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    y_ws = wf_gpu.das(scan, rf, workspace=ws)
    y_plain = wf_gpu.das(scan, rf, workspace=torch.empty(0, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    iz = np.repeat(np.arange(w.nz), w.nx).reshape(w.nz, w.nx)
    ix = np.tile(np.arange(w.nx), (w.nz, 1))
    ref = oracle.das_workload(rf_np[0].astype(np.float64), w, iz, ix)
    # deepest row any echo inside the record can reach: the two-way path is
    # at least z (1 + cos 10 deg), in samples, and must stay below S - 1
    zs = np.linspace(w.z_min, w.z_max, w.nz) * w.fs / w.c
    dead = zs * (1.0 + math.cos(math.radians(10.0))) > w.n_s
    assert dead.any() and not dead.all()
    for y in (y_ws, y_plain):
        yc = y[0].cpu().numpy().astype(np.float64)
        err = nl2(yc, ref)
        print(f"deep grid: nL2 {err:.2e}, dead rows {int(dead.sum())}")
        assert err <= NL2_TOL
        assert np.all(yc[dead] == 0.0)


@pytest.mark.oracle_frames("pwi", "stai_full")
@pytest.mark.parametrize("name", ["pwi", "stai_full"])
def test_full_frame_bmode(wf_gpu, name):
    """The whole full-size frame in the benchmark's launch configuration
    (its work-split workspace, a plan): beamformed RF against the oracle's
    whole frame, and the B-mode image against the oracle's, whose dB scale
    takes the frame maximum (the clip of Sec. III) - over every pixel."""
    import oracle_frames

    torch = _torch()
    w = phantom.get_workload(name)
    scan = scan_from_workload(w)
    plan = wf_gpu.Plan(scan, w.n_s)
    wsb = plan.workspace_bytes(1)[0]
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    rf = phantom.synth_rf(w)
    y = wf_gpu.das(scan, _gpu(rf), workspace=ws, plan=plan)
    b = wf_gpu.bmode(y, w.dr_db)
    torch.cuda.synchronize()
    ref = oracle_frames.das_frame(w)
    b_ref = oracle.bmode(ref, w.dr_db)
    err = nl2(y[0].cpu().numpy(), ref)
    d = np.abs(b[0].cpu().numpy() - b_ref)
    print(f"{name} whole frame: DAS nL2 {err:.2e}, B-mode max |dB diff| {d.max():.2e} "
          f"(p99 {np.percentile(d, 99):.1e}), split workspace {wsb} bytes")
    assert err <= NL2_TOL
    assert d.max() <= DB_TOL
