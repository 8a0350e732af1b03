"""Precision of RF storage (int16 ADC counts, FP16) with FP32 accumulation,
against the FP64 oracle, on an 8-frame PWI batch (the PWI geometry: 64
plane waves x 128 channels x 2048 samples, 1024 x 512 grid).

Two errors are stated per frame:
  kernel error   GPU vs oracle fed exactly the stored values  (<= 1e-5 nL2)
  storage error  GPU vs oracle fed the unquantised float64 record
                 (<= 1e-3 nL2 for int16 and FP16 storage)
FP16 storage holds the int16 counts scaled by 2^-13 (|x| < 1), since FP16
represents integers exactly only up to 2048.  The oracle runs on whole
sampled columns of every frame.
"""

import numpy as np
import pytest

import oracle
import phantom
from phantom.prepare import lighter
from wfhelp import nl2, scan_from_workload

pytestmark = pytest.mark.gpu

COLS = (3, 170, 341, 508)
FP16_SCALE = 2.0 ** -13


def _batch_workload():
    return lighter(phantom.get_workload("pwi_batch8"))


def _cols(w):
    iz = np.repeat(np.arange(w.nz), len(COLS)).reshape(w.nz, len(COLS))
    ix = np.tile(np.asarray(COLS), (w.nz, 1))
    return iz, ix


def test_batch8_int16_and_fp16_storage(wf_gpu):
    import torch

    w = _batch_workload()
    rf_i16 = phantom.synth_rf(w)                    # [8][64][128][2048] int16
    rf_f64 = phantom.synth_rf(w, quantize=False)    # same record before rounding
    assert rf_i16.shape[0] == 8
    rf_f16 = (rf_i16.astype(np.float32) * FP16_SCALE).astype(np.float16)
    scan = scan_from_workload(w.with_(n_frames=1))
    y16 = wf_gpu.das(scan, torch.from_numpy(rf_i16).cuda())
    yh = wf_gpu.das(scan, torch.from_numpy(rf_f16).cuda())
    torch.cuda.synchronize()
    y16 = y16.cpu().numpy()
    yh = yh.cpu().numpy() / FP16_SCALE
    iz, ix = _cols(w)
    w1 = w.with_(n_frames=1)
    rows = []
    for f in range(8):
        ref_i16 = oracle.das_workload(rf_i16[f].astype(np.float64), w1, iz, ix)
        ref_f16 = oracle.das_workload(rf_f16[f].astype(np.float64), w1, iz, ix) / FP16_SCALE
        ref_f64 = oracle.das_workload(rf_f64[f], w1, iz, ix)
        g16 = y16[f][:, list(COLS)]
        gh = yh[f][:, list(COLS)]
        r = dict(frame=f, kernel_i16=nl2(g16, ref_i16), kernel_f16=nl2(gh, ref_f16),
                 storage_i16=nl2(g16, ref_f64), storage_f16=nl2(gh, ref_f64))
        rows.append(r)
        print("frame {frame}: kernel int16 {kernel_i16:.2e} fp16 {kernel_f16:.2e} | "
              "vs unquantised int16 {storage_i16:.2e} fp16 {storage_f16:.2e}".format(**r))
    for r in rows:
        assert r["kernel_i16"] <= 1e-5 and r["kernel_f16"] <= 1e-5
        assert r["storage_i16"] <= 1e-3 and r["storage_f16"] <= 1e-3
    # the batch call equals per-frame calls bit for bit
    one = wf_gpu.das(scan, torch.from_numpy(rf_i16[5]).cuda()).cpu().numpy()
    assert np.array_equal(one, y16[5])
