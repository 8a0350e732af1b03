"""Derivatives of DAS on the GPU, through the C ABI, against the FP64 oracle.

  adjoint w.r.t. RF   vs oracle transpose: nL2 <= 1e-5 (the cotangent is
                      rounded to 24 bits of its frame maximum; sums are exact
                      integers, so two runs agree bit for bit)
  dot-product test    <A r, g> = <r, A^T g> with both GPU kernels: rel 1e-5
  d y / d c           vs oracle: nL2 <= 1e-5 on a smooth record; on speckle
                      the derivative of the piecewise-linear interpolant jumps
                      where u crosses an integer, and a ~1e-7-sample delay
                      difference moves a crossing with probability ~1e-7 per
                      term, so the bar there is 2e-3 (a few pixels change one
                      of their 8192 terms)
  d L / d c           GPU analytic vs oracle analytic: rel 2e-3 (kinks); the
                      central finite difference (h = 0.5 m/s) of the GPU
                      forward on the 64 x 64 sub-grid equals the mean of the
                      analytic derivative over [c - h, c + h]: rel 2e-2
"""

import numpy as np
import pytest

import oracle
import phantom
from phantom.configs import subgrid
from phantom.prepare import lighter
from wfhelp import deep_pwi, nl2, scan_from_workload

pytestmark = pytest.mark.gpu


def _t():
    import torch

    return torch


CASES = {
    "tiny_stai_apod_t0": lambda: phantom.tiny_stai(f_number=0.8, t0=0.3e-6),
    "tiny_pwi_apod": lambda: phantom.tiny_pwi(f_number=1.2, t0=-0.2e-6, tref="centre"),
    "pwi_sub": lambda: subgrid(phantom.get_workload("pwi").with_(n_tx=8, angles_deg=tuple(
        np.linspace(-16, 16, 8))), 300, 70, 200, 20),
    # split into items, with items that run nothing left out of the work list
    "stai_small": lambda: phantom.get_workload("stai_small"),
    "deep_pwi": deep_pwi,
    # the gather runs 512 x 2 tiles, the adjoint its own 1024 x 1 tiles,
    # split and work list
    "stai_own_tiles": lambda: subgrid(lighter(phantom.get_workload("stai_full"), 2000).with_(
        n_tx=16), 64, 128, 40, 64),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_matches_oracle_and_dot_product(wf_gpu, name):
    torch = _t()
    w = CASES[name]()
    if name in ("stai_small", "deep_pwi"):
        info = wf_gpu.tile_info(scan_from_workload(w), w.n_s)
        assert info["workgroups"] < info["ntz"] * info["ntx"] * info["nsplit"]
    if name == "stai_own_tiles":
        info = wf_gpu.tile_info(scan_from_workload(w), w.n_s)
        assert (info["threads"], info["px"]) == (512, 2)
        assert (info["adjoint_threads"], info["adjoint_px"]) == (1024, 1)
        assert info["adjoint_nsplit"] > 1
    rng = np.random.default_rng(4)
    g = rng.normal(size=(w.nz, w.nx)).astype(np.float32)
    r = rng.normal(size=(w.n_tx, w.n_ch, w.n_s)).astype(np.float32)
    scan = scan_from_workload(w)
    gr = wf_gpu.das_adjoint(scan, torch.from_numpy(g).cuda()[None], w.n_s)
    gr2 = wf_gpu.das_adjoint(scan, torch.from_numpy(g).cuda()[None], w.n_s)
    y = wf_gpu.das(scan, torch.from_numpy(r).cuda()[None])
    torch.cuda.synchronize()
    assert torch.equal(gr, gr2)  # bitwise reproducible
    ref = oracle.das_adjoint_workload(g.astype(np.float64), w)
    err = nl2(gr[0].cpu().numpy(), ref)
    lhs = float(np.sum(y[0].cpu().numpy().astype(np.float64) * g))
    rhs = float(np.sum(r.astype(np.float64) * gr[0].cpu().numpy()))
    print(f"{name}: adjoint nL2 {err:.2e}, dot-product rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert err <= 1e-5
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_adjoint_full_size_production_launch(wf_gpu):
    """The adjoint of the full PWI frame (1024 x 512, 64 plane waves x 128
    channels x 2048 samples) in its production launch: unsplit 1024-thread
    tiles, two window sets, the 1.7 GB per-tile window workspace and the
    stage-2 reduce over all 256 tiles.  The cotangent is non-zero on four
    whole columns, whose transpose the oracle computes; every sample of the
    [T][C][S] gradient is compared, and the dot-product identity ties it to
    the forward gather at the same size."""
    torch = _t()
    w = phantom.get_workload("pwi")
    scan = scan_from_workload(w)
    info = wf_gpu.tile_info(scan, w.n_s, 1, 2)
    assert info["threads"] == 1024 and info["nsplit"] == 1
    assert info["workgroups"] == info["ntz"] * info["ntx"] == 256
    plan = wf_gpu.Plan(scan, w.n_s)
    adj_bytes = plan.workspace_bytes(1)[1]
    assert adj_bytes > (1 << 30)
    cols = np.array([0, 131, 256, 511])
    rng = np.random.default_rng(17)
    gc = rng.normal(size=(w.nz, len(cols)))
    g = np.zeros((w.nz, w.nx), dtype=np.float32)
    g[:, cols] = gc.astype(np.float32)
    ws = torch.empty(adj_bytes, dtype=torch.uint8, device="cuda")
    gr = wf_gpu.das_adjoint(scan, torch.from_numpy(g).cuda()[None], w.n_s, workspace=ws,
                            plan=plan)
    r = phantom.synth_rf(w)[0].astype(np.float32)
    y = wf_gpu.das(scan, torch.from_numpy(r).cuda()[None], plan=plan)
    torch.cuda.synchronize()
    iz = np.repeat(np.arange(w.nz), len(cols)).reshape(w.nz, len(cols))
    ix = np.tile(cols, (w.nz, 1))
    ref = oracle.das_adjoint_workload(g[:, cols].astype(np.float64), w, iz, ix)
    got = gr[0].cpu().numpy()
    err = nl2(got, ref)
    lhs = float(np.sum(y[0].cpu().numpy().astype(np.float64)[:, cols] * g[:, cols]))
    rhs = float(np.sum(r.astype(np.float64) * got))
    print(f"pwi full adjoint: nL2 {err:.2e} over {got.size} samples, dot-product rel "
          f"{abs(lhs - rhs) / abs(lhs):.2e}, workspace {adj_bytes / 2**30:.2f} GiB")
    assert err <= 1e-5
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def _smooth_rf(w, seed=5):
    rng = np.random.default_rng(seed)
    s = np.arange(w.n_s)
    ph = rng.uniform(0, 2 * np.pi, size=(w.n_tx, w.n_ch, 1))
    return (1000.0 * np.cos(2 * np.pi * 0.01 * s[None, None, :] + ph)).astype(np.float32)


def test_dydc_matches_oracle(wf_gpu):
    torch = _t()
    w = CASES["pwi_sub"]()
    scan = scan_from_workload(w)
    for kind, rf, bar in (("smooth", _smooth_rf(w), 1e-5),
                          ("speckle", phantom.synth_rf(lighter(w.with_(nz=1024, nx=512,
                                                                       z_min=5e-3,
                                                                       z_max=30e-3,
                                                                       x_min=None,
                                                                       x_max=None)))[0]
                           .astype(np.float32), 2e-3)):
        d = wf_gpu.das_dydc(scan, torch.from_numpy(rf).cuda()[None])
        torch.cuda.synchronize()
        ref = oracle.das_dydc_workload(rf.astype(np.float64), w)
        err = nl2(d[0].cpu().numpy(), ref)
        print(f"dy/dc {kind}: nL2 {err:.2e}")
        assert err <= bar


@pytest.mark.parametrize("c", [1480.0, 1540.0, 1600.0])
def test_dldc_finite_difference_and_oracle(wf_gpu, c):
    """PWI geometry, 64 x 64 sub-grid at the image centre, L = <g, y>.

    With h = 0.5 m/s every delay moves by ~0.67 samples, a large step for
    9-samples-per-period RF, so the central difference is compared with what
    it exactly equals - the mean of dL/dc over [c - h, c + h] (L is
    continuous in c) - integrated from the analytic derivative by the
    trapezoid rule on 65 points; the gap to the point derivative is only
    reported.  GPU vs oracle analytic: the kink crossings (see module
    docstring) bound the agreement to ~1e-3 of the scalar."""
    torch = _t()
    base = lighter(phantom.get_workload("pwi"))
    rf = phantom.synth_rf(base)[0].astype(np.float32)  # synthesised at 1540 m/s
    w = subgrid(base, 480, 64, 224, 64).with_(c=c)
    rng = np.random.default_rng(7)
    g = rng.normal(size=(w.nz, w.nx)).astype(np.float32)
    rf_t = torch.from_numpy(rf).cuda()[None]
    g_t = torch.from_numpy(g).cuda()

    def dldc(cc):
        dydc = wf_gpu.das_dydc(scan_from_workload(w.with_(c=cc)), rf_t)
        return float(wf_gpu.dot(g_t.reshape(-1), dydc.reshape(-1)).item())

    dl = dldc(c)
    h = 0.5
    ys = [wf_gpu.das(scan_from_workload(w.with_(c=c + s * h)), rf_t) for s in (1, -1)]
    fd = float(((ys[0] - ys[1]) * g_t).double().sum().item()) / (2 * h)
    cs = np.linspace(c - h, c + h, 65)
    vals = np.array([dldc(float(x)) for x in cs])
    mean = float(np.sum((vals[1:] + vals[:-1]) * 0.5) / (len(cs) - 1))
    ref = float(np.sum(g.astype(np.float64) * oracle.das_dydc_workload(rf.astype(np.float64), w)))
    print(f"c={c}: dL/dc gpu {dl:.6e} oracle {ref:.6e} | fd(h=0.5) {fd:.6e} vs mean of the "
          f"analytic over [c-h, c+h] {mean:.6e} (rel {abs(fd - mean) / abs(fd):.2e}); "
          f"point derivative vs fd rel {abs(dl - fd) / abs(fd):.2e}")
    assert abs(dl - ref) <= 2e-3 * abs(ref)
    assert abs(fd - mean) <= 0.02 * abs(fd)


def test_autograd_function(wf_gpu):
    torch = _t()
    w = CASES["pwi_sub"]()
    scan = scan_from_workload(w)
    rng = np.random.default_rng(8)
    rf = torch.from_numpy(rng.normal(size=(1, w.n_tx, w.n_ch, w.n_s)).astype(np.float32)).cuda()
    rf.requires_grad_(True)
    c = torch.tensor(w.c, dtype=torch.float32, device="cuda", requires_grad=True)
    g = torch.from_numpy(rng.normal(size=(1, w.nz, w.nx)).astype(np.float32)).cuda()
    y = wf_gpu.das_autograd(scan, rf, c)
    (y * g).sum().backward()
    gr = wf_gpu.das_adjoint(scan, g, w.n_s)
    dydc = wf_gpu.das_dydc(scan, rf.detach())
    dl = wf_gpu.dot(g.reshape(-1), dydc.reshape(-1))
    torch.cuda.synchronize()
    assert nl2(rf.grad.cpu().numpy(), gr.cpu().numpy()) <= 1e-6
    assert abs(float(c.grad) - float(dl)) <= 1e-6 * abs(float(dl))


def test_adjoint_workspace_and_frames(wf_gpu):
    """A short workspace is refused with WF_ERR_WORKSPACE; a two-frame call
    equals the two one-frame calls (the workspace is reused frame by frame)."""
    torch = _t()
    w = CASES["pwi_sub"]()
    scan = scan_from_workload(w)
    need = wf_gpu.adjoint_workspace_bytes(scan, w.n_s)
    assert need > 0
    rng = np.random.default_rng(12)
    g = torch.from_numpy(rng.normal(size=(2, w.nz, w.nx)).astype(np.float32)).cuda()
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(wf_gpu.WfError) as ei:
        wf_gpu.das_adjoint(scan, g, w.n_s, workspace=small)
    assert ei.value.status == -4
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    both = wf_gpu.das_adjoint(scan, g, w.n_s, workspace=ws)
    f0 = wf_gpu.das_adjoint(scan, g[0], w.n_s, workspace=ws)
    f1 = wf_gpu.das_adjoint(scan, g[1], w.n_s, workspace=ws)
    torch.cuda.synchronize()
    for a, b in ((both[0], f0[0]), (both[1], f1[0])):
        assert nl2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("op", ["das", "dydc"])
def test_int16_rf_matches_float_rf_on_large_tiles(wf_gpu, op):
    """int16 counts convert to float exactly and are staged the same way, so
    the same integer RF given as int16 and as float32 gives the same bits.
    On 1024-thread tiles the int16 gather stages two passes per barrier and
    the float32 one a single pass, so this also pins the two pipelines to
    each other."""
    torch = _t()
    w = subgrid(lighter(phantom.get_workload("pwi")), 300, 128, 200, 96).with_(phantom="random")
    info = wf_gpu.tile_info(scan_from_workload(w), w.n_s, 1)
    assert info["threads"] == 1024
    rf = phantom.synth_rf(w)[0]
    scan = scan_from_workload(w)
    fn = wf_gpu.das if op == "das" else wf_gpu.das_dydc
    r16 = torch.from_numpy(rf).cuda()[None]
    r32 = torch.from_numpy(rf.astype(np.float32)).cuda()[None]
    a = fn(scan, r16)
    b = fn(scan, r32)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.abs(b).max() > 0
    assert np.array_equal(a, b)
