"""Plans on the GPU: calls with a plan equal calls without one bit for bit;
the first call of a never-seen geometry, made with a plan, is captured into a
HIP graph and every replay matches the FP64 oracle; learning the speed of
sound through the autograd wrapper adds nothing to the library's cache.

Bars: beamformed RF nL2 <= 1e-5 and B-mode within 0.01 dB of the oracle;
plan vs no plan bitwise (same kernels, same tables)."""

import numpy as np
import pytest

import oracle
import phantom
from phantom.configs import subgrid
from phantom.prepare import lighter
from wfhelp import nl2, scan_from_workload

pytestmark = pytest.mark.gpu


def _t():
    import torch

    return torch


@pytest.mark.parametrize("name", ["stai_small", "pwi_sub", "deep_pwi"])
def test_plan_equals_no_plan(wf_gpu, name):
    """Forward, d y / d c and adjoint with a plan give the bits of the same
    calls without one (split workspace, work list and plain tile order)."""
    from wfhelp import deep_pwi

    torch = _t()
    if name == "stai_small":
        w = phantom.get_workload("stai_small")
    elif name == "pwi_sub":
        w = subgrid(lighter(phantom.get_workload("pwi")), 300, 128, 200, 96)
    else:
        w = deep_pwi()
    scan = scan_from_workload(w)
    rf = torch.from_numpy(phantom.synth_rf(w)).cuda()
    plan = wf_gpu.Plan(scan, w.n_s)
    a = wf_gpu.das(scan, rf, plan=plan)
    b = wf_gpu.das(scan, rf)
    rf32 = rf.float()
    da = wf_gpu.das_dydc(scan, rf32, plan=plan)
    db = wf_gpu.das_dydc(scan, rf32)
    g = torch.randn(a.shape, generator=torch.Generator(device="cuda").manual_seed(5),
                    device="cuda")
    ga = wf_gpu.das_adjoint(scan, g, w.n_s, plan=plan)
    gb = wf_gpu.das_adjoint(scan, g, w.n_s)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(da, db) and torch.equal(ga, gb)
    ref = oracle.das_workload(phantom.synth_rf(w)[0].astype(np.float64), w)
    assert nl2(a[0].cpu().numpy(), ref) <= 1e-5


def _table_cases():
    """Geometries over every tile shape and delay path: STAI small (512 x 1
    tiles, split, work list), STAI with t0 != 0 and an f-number (transmit
    delays with a time origin, apodised receive words), a STAI sub-grid on
    512 x 2 tiles, a coarse 256 x 128 STAI grid (256 x 1 tiles), PWI
    sub-grid (1024 x 2 tiles, two passes per barrier), PWI deeper than its
    record, and the full 1024 x 512 PWI frame (1024 x 2 tiles; its oracle
    parity is the full-frame test's)."""
    from phantom.configs import served_mix
    from wfhelp import deep_pwi

    full = lighter(phantom.get_workload("stai_full"), 2000)
    coarse = next(w for w in served_mix() if w.name == "stai_n128_t16_s1024_256x128")
    return {
        "stai_small": phantom.get_workload("stai_small"),
        # (no pixel lies within 1e-4 of an aperture edge: at an exact tie
        # 2 F# |x - x_j| = z, float rounding decides either way)
        "stai_t0_fnum": phantom.tiny_stai(n_elem=32, n_tx=32, n_ch=32, n_s=1024, nz=96, nx=40,
                                          z_min=4.05e-3, z_max=11.9e-3, f_number=1.17,
                                          t0=0.35e-6),
        "stai_full_sub": subgrid(full.with_(n_tx=48), 64, 192, 40, 96),
        "stai_coarse": coarse,
        "pwi_sub": subgrid(lighter(phantom.get_workload("pwi")), 300, 128, 200, 96),
        "deep_pwi": deep_pwi(),
        "pwi_full": lighter(phantom.get_workload("pwi")),
    }


@pytest.mark.parametrize("name", ["stai_small", "stai_t0_fnum", "stai_full_sub", "stai_coarse",
                                  "pwi_sub", "deep_pwi", "pwi_full"])
def test_delay_tables_give_the_same_bits(wf_gpu, name):
    """A plan with the delay tables (the gathers read the receive and STAI
    transmit words) and one without (the gathers form them) give the same
    bits: single frames with and without the split workspace, a batch of
    three frames (frame groups), FP32 RF and d y / d c; and the oracle's
    result within 1e-5."""
    torch = _t()
    w = _table_cases()[name]
    scan = scan_from_workload(w)
    rf_np = phantom.synth_rf(w)
    rf = torch.from_numpy(rf_np).cuda()
    with_t = wf_gpu.Plan(scan, w.n_s, delay_tables=True)
    without = wf_gpu.Plan(scan, w.n_s, delay_tables=False)
    assert with_t.mem.numel() > without.mem.numel()
    outs = {}
    for key, plan in (("tables", with_t), ("plain", without)):
        wsb = plan.workspace_bytes(3)[0]
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda") if wsb else None
        rf3 = rf.repeat(3, 1, 1, 1)
        rf3[1] = torch.roll(rf[0], 7, dims=-1)
        rf3[2] = -rf[0]
        outs[key] = (wf_gpu.das(scan, rf, plan=plan, workspace=ws),
                     wf_gpu.das(scan, rf, plan=plan),
                     wf_gpu.das(scan, rf3, plan=plan, workspace=ws),
                     wf_gpu.das(scan, rf.float(), plan=plan),
                     wf_gpu.das_dydc(scan, rf.float(), plan=plan))
    torch.cuda.synchronize()
    for a, b in zip(outs["tables"], outs["plain"]):
        assert torch.equal(a, b)
    if name == "pwi_full":
        return
    ref = oracle.das_workload(rf_np[0].astype(np.float64), w)
    err = nl2(outs["tables"][0][0].cpu().numpy(), ref)
    print(f"{name}: nL2 {err:.2e}")
    assert err <= 1e-5


def test_plan_of_another_geometry_is_refused(wf_gpu):
    torch = _t()
    w = phantom.get_workload("stai_small")
    scan = scan_from_workload(w)
    rf = torch.from_numpy(phantom.synth_rf(w)).cuda()
    other = scan_from_workload(w.with_(c=1500.0))
    plan = wf_gpu.Plan(other, w.n_s)
    with pytest.raises(wf_gpu.WfError) as ei:
        wf_gpu.das(scan, rf, plan=plan)
    assert ei.value.status == -1 and "another geometry" in str(ei.value)


def test_first_call_of_a_new_geometry_is_captured(wf_gpu):
    """A PWI geometry at a speed of sound no call has used: build its plan,
    then capture DAS -> envelope -> log compression into a graph without
    any eager call first.  Replays, with eager work of the program and
    synchronisations between them, each match the oracle."""
    torch = _t()
    w = subgrid(lighter(phantom.get_workload("pwi")), 400, 128, 150, 96)
    w_rf = w
    w = w.with_(c=1537.3125)  # beamform at a c never seen before (RF from 1540)
    scan = scan_from_workload(w)
    rf_np = phantom.synth_rf(w_rf)
    rf = torch.from_numpy(rf_np).cuda()
    before = wf_gpu.geometry_cache_info()
    plan = wf_gpu.Plan(scan, w.n_s)
    ws_bytes = plan.workspace_bytes(1)[0]
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    y = torch.empty((1, w.nz, w.nx), dtype=torch.float32, device="cuda")
    out = torch.empty_like(y)
    col_max = torch.empty((1, w.nx), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        wf_gpu.das(scan, rf, out=y, workspace=ws, plan=plan)
        wf_gpu.bmode(y, w.dr_db, out=out, col_max=col_max)
    torch.cuda.synchronize()
    assert wf_gpu.geometry_cache_info() == before
    ref = oracle.das_workload(rf_np[0].astype(np.float64), w)
    b_ref = oracle.bmode(ref, w.dr_db)
    scratch = torch.randn(1 << 20, device="cuda")
    for k in range(3):
        y.fill_(float("nan"))
        out.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        err = nl2(y[0].cpu().numpy(), ref)
        d = float(np.max(np.abs(out[0].cpu().numpy() - b_ref)))
        print(f"replay {k}: nL2 {err:.2e}, max |dB diff| {d:.2e}")
        assert err <= 1e-5 and d <= 0.01
        scratch.mul_(1.5).add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
    eager = wf_gpu.das(scan, rf, plan=plan)
    torch.cuda.synchronize()
    assert torch.equal(eager, y)


def test_learning_c_adds_nothing_to_the_cache(wf_gpu):
    """The autograd wrapper at 12 distinct speeds of sound: forward and
    backward (RF and c gradients) run with one plan per c in torch memory;
    the library's cache does not grow, and the gradient w.r.t. c at each c
    matches the oracle's analytic derivative."""
    torch = _t()
    w = phantom.tiny_pwi(n_elem=32, n_ch=32, n_tx=6, n_s=1024, nz=96, nx=40, z_min=6e-3,
                         z_max=11e-3, phantom="random",
                         angles_deg=(-12.0, -7.0, -2.0, 0.0, 5.0, 9.0))
    base = scan_from_workload(w)
    rf_np = phantom.synth_rf(w)[0].astype(np.float32)
    rng = np.random.default_rng(4)
    g_np = rng.normal(size=(w.nz, w.nx))
    before = wf_gpu.geometry_cache_info()
    for c in np.linspace(1490.0, 1590.0, 12):
        rf = torch.from_numpy(rf_np).cuda().requires_grad_(True)
        ct = torch.tensor(float(c), dtype=torch.float64, requires_grad=True)
        y = wf_gpu.das_autograd(base, rf, ct)
        loss = (y * torch.from_numpy(g_np).float().cuda()).sum()
        loss.backward()
        torch.cuda.synchronize()
        assert rf.grad is not None and ct.grad is not None
    assert wf_gpu.geometry_cache_info() == before
    # the last c against the oracle's analytic dL/dc (the dy/dc parity bars)
    wc = w.with_(c=float(c))
    ref = float(np.sum(g_np * oracle.das_dydc_workload(rf_np.astype(np.float64), wc)))
    got = float(ct.grad)
    rel = abs(got - ref) / abs(ref)
    print(f"dL/dc at c={c:.1f}: {got:.6e} vs oracle {ref:.6e} (rel {rel:.2e})")
    assert rel <= 2e-3
