"""wf_das_noalloc (the DAS entry point that allocates nothing: geometry
tables and split partial frames in a static per-GPU scratch array) against
wf_das_stai / wf_das_pwi, through the C ABI, on an MI355X.

Calls run back to back on one stream, each later one on a smaller input, so
a call that read the previous call's tables or partial frames from the
shared scratch would show.  Bars: bitwise equal where both calls run the
same split (the same kernels and summation order); the normalised L2 bar of
the beamformed RF (1e-5) where the scratch is too small for the partial
frames and the call runs unsplit; and the FP64 oracle on the last call."""

import numpy as np
import pytest

import oracle
import phantom
from wfhelp import nl2, scan_from_workload

pytestmark = pytest.mark.gpu


def _cases():
    big = phantom.get_workload("stai_small")
    small = phantom.tiny_pwi(n_elem=32, n_ch=32, n_tx=6, n_s=1024, nz=96, nx=40, z_min=6e-3,
                             z_max=11e-3, angles_deg=(-12.0, -7.0, -2.0, 0.0, 5.0, 9.0))
    # (workload, frames): 40 frames of partials (20 MiB) exceed the scratch,
    # 2 frames fit beside the tables, the PWI grid is smaller still
    return [(big, 40), (big, 2), (small, 1)]


def test_noalloc_matches_the_allocating_entry_point(wf_gpu):
    import torch

    scratch = 16 << 20  # WF_NOALLOC_SCRATCH_BYTES
    outs = []
    for w, nf in _cases():
        scan = scan_from_workload(w)
        rf1 = phantom.synth_rf(w)[0]
        rf = torch.from_numpy(np.repeat(rf1[None], nf, axis=0)).cuda()
        ws = wf_gpu.das_workspace_bytes(scan, w.n_s, nf)
        out = torch.full((nf, w.nz, w.nx), float("nan"), device="cuda")
        y = wf_gpu.das_noalloc(scan, rf, out=out)
        ref = wf_gpu.das(scan, rf)  # wf_das_stai / wf_das_pwi with a workspace
        fits = 0 < ws and ws + (64 << 10) <= scratch
        outs.append((w, nf, y, ref, fits, rf1))
    torch.cuda.synchronize()
    for w, nf, y, ref, fits, rf1 in outs:
        assert not torch.isnan(y).any(), f"{w.name} x{nf}: unwritten pixels"
        err = nl2(y.cpu().numpy(), ref.cpu().numpy())
        same = bool(torch.equal(y, ref))
        print(f"{w.name} x{nf}: split partials in scratch {fits}, nL2 vs wf_das_* {err:.2e}, "
              f"bitwise {same}")
        assert err <= 1e-5
        if fits:
            assert same
    # the last (smallest) call against the oracle
    w, nf, y, _, _, rf1 = outs[-1]
    y_ref = oracle.das_workload(rf1.astype(np.float64), w)
    err = nl2(y[0].cpu().numpy(), y_ref)
    print(f"{w.name}: nL2 vs oracle {err:.2e}")
    assert err <= 1e-5
