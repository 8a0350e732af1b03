"""FIR pre-filter and qUS moment maps on the GPU, through the C ABI, against
the FP64 oracle.

Bars (FP32 fused multiply-adds / sums in a fixed order; the inputs the
oracle sees are exactly the values the kernels read):
  FIR       normalised L2 <= 2e-6 per case; an impulse returns the taps
            bit-exactly; records never leak into each other.
  moments   per element relative <= 3e-5 (positive sums of <= wz + wx
            sequential FP32 additions), normalised L2 <= 2e-6 per map.
  pipeline  FIR -> DAS -> envelope -> moments vs the oracle chain:
            normalised L2 <= 1e-5 per map.
"""

import numpy as np
import pytest

import oracle
import phantom
from phantom.configs import FIR_TAPS, QUS_WINDOW
from wfhelp import nl2, scan_from_workload

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


@pytest.mark.parametrize("dtype", ["int16", "float16", "float32"])
@pytest.mark.parametrize("k_len", [1, 7, 15, 21, 31, 45, 63])
def test_fir_matches_oracle(wf_gpu, dtype, k_len):
    torch = _torch()
    rng = np.random.default_rng(100 + k_len)
    taps = rng.normal(size=k_len).astype(np.float32)
    for n_rec, n_s in ((37, 1024), (5, 2056), (300, 8), (3, 64), (1, 4096)):
        if dtype == "int16":
            r = rng.integers(-8191, 8192, size=(n_rec, n_s)).astype(np.int16)
        elif dtype == "float16":
            r = (rng.integers(-8191, 8192, size=(n_rec, n_s)) * 2.0 ** -13).astype(np.float16)
        else:
            r = rng.normal(size=(n_rec, n_s)).astype(np.float32)
        y = wf_gpu.fir(torch.from_numpy(r).cuda(), taps)
        torch.cuda.synchronize()
        ref = oracle.fir_same(r.astype(np.float64), taps.astype(np.float64))
        err = nl2(y.cpu().numpy(), ref)
        assert err <= 2e-6, f"{dtype} K={k_len} {n_rec}x{n_s}: nL2 {err:.2e}"


def test_fir_impulse_and_record_edges(wf_gpu):
    torch = _torch()
    taps = np.random.default_rng(7).normal(size=63).astype(np.float32)
    n_s = 128
    r = np.zeros((4, n_s), dtype=np.float32)
    r[1, 64] = 1.0  # interior impulse of record 1
    r[2, 0] = 1.0   # impulses at record edges: the neighbours must stay zero
    r[2, n_s - 1] = 1.0
    y = wf_gpu.fir(torch.from_numpy(r).cuda(), taps).cpu().numpy()
    exp = np.zeros_like(r)
    exp[1, 64 - 31:64 + 32] = taps
    exp[2, :32] = taps[31:]
    exp[2, n_s - 32:] = taps[:32]
    assert np.array_equal(y, exp)


def test_fir_edge_cases(wf_gpu):
    torch = _torch()
    taps = np.array([0.25, 0.5, 0.25], dtype=np.float32)
    empty = torch.zeros((0, 64), dtype=torch.int16, device="cuda")
    assert wf_gpu.fir(empty, taps).shape == (0, 64)
    x = torch.arange(16, dtype=torch.float32, device="cuda").reshape(2, 8)
    one = wf_gpu.fir(x, [1.0])
    assert torch.equal(one, x)
    with pytest.raises(wf_gpu.WfError):
        wf_gpu.fir(x, [1.0, 2.0])  # even tap count
    with pytest.raises(wf_gpu.WfError):
        wf_gpu.fir(torch.zeros((2, 12), device="cuda"), taps)  # n_s % 8 != 0
    with pytest.raises(wf_gpu.WfError):
        wf_gpu.fir(x, np.ones(65, dtype=np.float32))  # too many taps


def test_fir_full_pwi_sampled_records(wf_gpu):
    """The full PWI RF (64 x 128 x 2048 int16) in one launch; 64 sampled
    records against the oracle."""
    torch = _torch()
    w = phantom.get_workload("pwi")
    rf = phantom.synth_rf(w)
    taps = phantom.workload_taps(w, FIR_TAPS)
    y = wf_gpu.fir(torch.from_numpy(rf).cuda(), taps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    flat_in = rf.reshape(-1, w.n_s)
    flat_out = y.reshape(-1, w.n_s)
    idx = np.sort(rng.choice(flat_in.shape[0], 64, replace=False))
    got = flat_out[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = oracle.fir_same(flat_in[idx].astype(np.float64), taps.astype(np.float64))
    assert nl2(got, ref) <= 2e-6


@pytest.mark.parametrize("win", [(16, 8, 4, 2), (1, 1, 1, 1), (128, 96, 1, 1), (5, 3, 7, 11),
                                 (32, 8, 8, 2)])
def test_moments_match_oracle(wf_gpu, win):
    torch = _torch()
    wz, wx, sz, sx = win
    env = np.random.default_rng(11).rayleigh(100.0, size=(2, 128, 96)).astype(np.float32)
    got = wf_gpu.moments(torch.from_numpy(env).cuda(), wz, wx, sz, sx).cpu().numpy()
    ref = oracle.moment_maps(env.astype(np.float64), wz, wx, sz, sx)
    assert got.shape == ref.shape
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= 3e-5, f"{win}: max rel {rel:.2e}"
    for p in range(3):
        assert nl2(got[:, p], ref[:, p]) <= 2e-6


def test_moments_constant_and_errors(wf_gpu):
    torch = _torch()
    env = torch.full((1, 40, 30), 2.0, device="cuda")
    m = wf_gpu.moments(env, 8, 5, 4, 5)
    exp = torch.tensor([2.0, 4.0, 8.0], device="cuda")[None, :, None, None].expand_as(m)
    assert torch.equal(m, exp)
    with pytest.raises(ValueError):
        wf_gpu.moments(env, 41, 5, 1, 1)


def test_prefilter_to_moments_pipeline(wf_gpu):
    """FIR -> DAS (float32 RF) -> envelope -> moment maps on the small STAI
    workload, against the oracle chain."""
    torch = _torch()
    w = phantom.get_workload("stai_small")
    rf = phantom.synth_rf(w)
    taps = phantom.workload_taps(w, FIR_TAPS)
    q = dict(QUS_WINDOW, wz=16, sz=4)
    rf_f = wf_gpu.fir(torch.from_numpy(rf).cuda(), taps)
    y = wf_gpu.das(scan_from_workload(w), rf_f)
    env, _ = wf_gpu.envelope(y)
    m = wf_gpu.moments(env, q["wz"], q["wx"], q["sz"], q["sx"])
    torch.cuda.synchronize()
    rf64 = oracle.fir_same(rf.astype(np.float64)[0], taps.astype(np.float64))
    ref = oracle.moment_maps(oracle.envelope(oracle.das_workload(rf64, w)), q["wz"], q["wx"],
                             q["sz"], q["sx"])
    got = m[0].cpu().numpy()
    for p in range(3):
        err = nl2(got[p], ref[p])
        print(f"pipeline moment {p + 1}: nL2 {err:.2e}")
        assert err <= 1e-5
