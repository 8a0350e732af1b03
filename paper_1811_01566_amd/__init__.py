"""MI355X-native DAS -> envelope -> B-mode path (WaveFlow, arXiv 1811.01566).

Thin Python binding over ``libwf.so`` (C ABI in ``include/wf.h``): it
marshals arguments and passes torch device pointers and the current HIP
stream; every step of the path runs in the library's HIP kernels.  There is
no CPU fallback: calls fail when the library is missing or the tensors are
not on a GPU.

Pipeline (paper Fig. 2): :func:`das_stai` / :func:`das_pwi` (Beamforming,
Sec. II-B) -> :func:`envelope` (Analytic Signal + Absolute Value) ->
:func:`log_compress` (Dynamic Adjustment, dB clip of Sec. III); :func:`bmode`
runs the last two.  Around it: :func:`fir` (the FIR pre-filter of the RF,
Sec. II-B) and :func:`moments` (windowed E[X], E[X^2], E[X^3] of the
envelope, the qUS estimator's inputs, Fig. 3).
"""

from __future__ import annotations

import ctypes
import dataclasses
from dataclasses import dataclass
from typing import Optional, Sequence

from . import _lib
from ._lib import WfError, load

__all__ = ["Grid", "Scan", "Plan", "das", "das_stai", "das_pwi", "delays", "envelope",
           "log_compress", "bmode", "load", "WfError", "abi_version", "geometry_cache_clear",
           "geometry_cache_info", "plan_bytes", "tile_info", "adjoint_workspace_bytes", "das_workspace_bytes",
           "das_dydc", "das_adjoint", "dot", "DASFunction", "das_autograd", "das_noalloc"]


@dataclass(frozen=True)
class Grid:
    """Pixel grid: pixel (iz, ix) at (x0 + ix*dx, z0 + iz*dz), metres."""
    nz: int
    nx: int
    z0: float
    dz: float
    x0: float
    dx: float


@dataclass(frozen=True)
class Scan:
    """Probe, transmit sequence and grid of one acquisition geometry.

    mode "stai": transmit t fires element tx_elem[t] (default t).
    mode "pwi": transmit t is a plane wave at angles_rad[t]; tref "first"
    (time zero when the first element fires) or "centre".
    """
    mode: str
    n_elem: int
    pitch: float
    c: float
    fs: float
    n_tx: int
    n_ch: int
    grid: Grid
    t0: float = 0.0
    f_number: float = 0.0
    tx_elem: Optional[Sequence[int]] = None
    angles_rad: Optional[Sequence[float]] = None
    tref: str = "first"
    rx_elem: Optional[Sequence[int]] = None
    elem_x: Optional[Sequence[float]] = None

    def das(self, rf, out=None, stream=None):
        return das(self, rf, out=out, stream=stream)


def abi_version() -> int:
    return int(load().wf_abi_version())


def geometry_cache_clear() -> None:
    """Free the library's cache behind calls made without a plan."""
    _lib.check(load().wf_geometry_cache_clear(), "wf_geometry_cache_clear")


def geometry_cache_info() -> tuple:
    """(geometries, device bytes) held by the cache behind calls made
    without a plan."""
    n, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _lib.check(load().wf_geometry_cache_info(ctypes.byref(n), ctypes.byref(b)),
               "wf_geometry_cache_info")
    return int(n.value), int(b.value)


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch

    return torch


def _stream_ptr(t, stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class _Keep:
    """Holds ctypes arrays alive for the duration of a call."""

    def __init__(self):
        self.items = []

    def arr(self, ctype, values):
        if values is None:
            return None
        a = (ctype * len(values))(*values)
        self.items.append(a)
        return ctypes.cast(a, ctypes.POINTER(ctype))


def _check_lengths(scan: Scan):
    """The library reads n_tx transmit entries, n_ch channel elements and
    n_elem element positions from these host lists: shorter ones would be
    read past their end."""
    for name, seq, n in (("tx_elem", scan.tx_elem, scan.n_tx),
                         ("angles_rad", scan.angles_rad, scan.n_tx),
                         ("rx_elem", scan.rx_elem, scan.n_ch),
                         ("elem_x", scan.elem_x, scan.n_elem)):
        if seq is not None and len(seq) != n:
            raise ValueError(f"scan.{name} has {len(seq)} entries, {n} expected")
    if scan.mode == "pwi" and scan.angles_rad is None:
        raise ValueError("a PWI scan needs angles_rad")


def _structs(scan: Scan, keep: _Keep, n_frames=1, n_s=0, dtype=0):
    _check_lengths(scan)
    probe = _lib.WfProbe(int(scan.n_elem), float(scan.pitch),
                         keep.arr(ctypes.c_double, scan.elem_x))
    acq = _lib.WfAcq(int(n_frames), int(scan.n_tx), int(scan.n_ch), int(n_s), int(dtype),
                     float(scan.c), float(scan.fs), float(scan.t0), float(scan.f_number),
                     keep.arr(ctypes.c_int32, scan.rx_elem))
    g = scan.grid
    grid = _lib.WfGrid(int(g.nz), int(g.nx), float(g.z0), float(g.dz), float(g.x0), float(g.dx))
    return probe, acq, grid


def _tref(scan):
    if scan.tref == "first":
        return _lib.WF_PWI_TREF_FIRST
    if scan.tref == "centre":
        return _lib.WF_PWI_TREF_CENTRE
    raise ValueError(f"tref must be 'first' or 'centre', got {scan.tref!r}")


def _rf_dtype(t):
    torch = _torch()
    m = {torch.int16: _lib.WF_RF_I16, torch.float16: _lib.WF_RF_F16,
         torch.float32: _lib.WF_RF_F32}
    if t.dtype not in m:
        raise TypeError(f"rf dtype {t.dtype} is not int16, float16 or float32")
    return m[t.dtype]


def _mode_args(scan: Scan, keep: _Keep):
    mode = 0 if scan.mode == "stai" else 1
    tx = keep.arr(ctypes.c_int32, scan.tx_elem) if mode == 0 else None
    ang = keep.arr(ctypes.c_double, scan.angles_rad) if mode == 1 else None
    tref = _tref(scan) if mode == 1 else 0
    return mode, tx, ang, tref


def _plan_flags(delay_tables: bool) -> int:
    return _lib.WF_PLAN_DELAY_TABLES if delay_tables else 0


def plan_bytes(scan: Scan, n_s: int, delay_tables: bool = True) -> int:
    """Device bytes of the :class:`Plan` of this scan and record length
    (host only)."""
    lib = load()
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, 1, n_s, _lib.WF_RF_I16)
    mode, tx, ang, tref = _mode_args(scan, keep)
    n = ctypes.c_uint64(0)
    flags = _plan_flags(delay_tables)
    if mode == 0:
        st = lib.wf_plan_bytes_stai(probe, acq, tx, grid, flags, ctypes.byref(n))
    else:
        st = lib.wf_plan_bytes_pwi(probe, acq, ang, tref, grid, flags, ctypes.byref(n))
    _lib.check(st, "wf_plan_bytes")
    return int(n.value)


class Plan:
    """Launch plan and device tables of one geometry (``scan`` with records
    of ``n_s`` samples) in caller-owned device memory, a uint8 tensor held
    by this object.  DAS, d y / d c and adjoint calls given the plan neither
    allocate nor synchronise, so they may be captured into HIP graphs.  The
    tables are written on ``stream`` (default: the device's current stream);
    calls on other streams must be ordered after it.  Keep the object alive
    while work that uses it may run (graph replays included).

    ``delay_tables`` (default) also stores the gathers' window-local delays
    of every pixel to every channel and from every transmit, formed once on
    the device (256 MiB for 128 channels on a 1024 x 512 PWI grid, whose
    gather forms its transmit delays itself): the DAS and d y / d c calls
    then skip forming them, with bitwise the same results."""

    def __init__(self, scan: Scan, n_s: int, device=None, stream=None,
                 delay_tables: bool = True):
        torch = _torch()
        lib = load()
        if scan.mode not in ("stai", "pwi"):
            raise ValueError(f"mode must be 'stai' or 'pwi', got {scan.mode!r}")
        self.scan, self.n_s, self._h = scan, int(n_s), None
        keep = _Keep()
        probe, acq, grid = _structs(scan, keep, 1, n_s, _lib.WF_RF_I16)
        mode, tx, ang, tref = _mode_args(scan, keep)
        flags = _plan_flags(delay_tables)
        self.delay_tables = bool(delay_tables)
        n = ctypes.c_uint64(plan_bytes(scan, n_s, delay_tables))
        dev = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.mem = torch.empty(int(n.value), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            sp = _stream_ptr(self.mem, stream)
            if mode == 0:
                st = lib.wf_plan_build_stai(probe, acq, tx, grid, flags,
                                            _dev(self.mem, "plan memory"), n.value,
                                            ctypes.byref(h), sp)
            else:
                st = lib.wf_plan_build_pwi(probe, acq, ang, tref, grid, flags,
                                           _dev(self.mem, "plan memory"), n.value,
                                           ctypes.byref(h), sp)
        _lib.check(st, "wf_plan_build")
        self._h = h
        self.device = dev

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("the plan was closed")
        return self._h

    def workspace_bytes(self, n_frames: int = 1) -> tuple:
        """(DAS / d y / d c split workspace for n_frames, adjoint workspace)."""
        d, a = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _lib.check(load().wf_plan_workspace(self.handle, int(n_frames), ctypes.byref(d),
                                            ctypes.byref(a)), "wf_plan_workspace")
        return int(d.value), int(a.value)

    def close(self):
        """Free the host handle (the device memory goes with the tensor)."""
        if self._h is not None and _lib._lib is not None:
            _lib._lib.wf_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def _plan_arg(plan, scan, n_s, device):
    if plan is None:
        return None
    if not isinstance(plan, Plan):
        raise TypeError("plan must be a Plan")
    if plan.n_s != n_s or plan.device != device:
        raise ValueError(f"plan was built for {plan.n_s} samples on {plan.device}, "
                         f"the call has {n_s} on {device}")
    return plan.handle


# ---------------------------------------------------------------------------
# public calls
# ---------------------------------------------------------------------------

def das_workspace_bytes(scan: Scan, n_s: int, n_frames: int = 1) -> int:
    """Bytes of the optional DAS workspace (0: the geometry never splits)."""
    lib = load()
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, n_frames, n_s, _lib.WF_RF_I16)
    mode, tx, ang, tref = _mode_args(scan, keep)
    n = ctypes.c_uint64(0)
    _lib.check(lib.wf_das_workspace(mode, probe, acq, tx, ang, tref, grid, ctypes.byref(n)),
               "wf_das_workspace")
    return int(n.value)


def _workspace_arg(scan, ns, nf, workspace, device, plan=None):
    """(pointer, bytes) of the DAS workspace: the caller's, or a fresh one
    when the geometry splits and none is given."""
    torch = _torch()
    if workspace is None:
        need = plan.workspace_bytes(nf)[0] if plan is not None else das_workspace_bytes(
            scan, ns, nf)
        if need == 0:
            return None, 0, None
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    return (_dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
            workspace)


def das(scan: Scan, rf, out=None, workspace=None, stream=None, plan: Optional[Plan] = None):
    """Delay-and-Sum of rf [F][T][C][S] (or [T][C][S]) -> float32 [F][nz][nx]
    (or [nz][nx]).  `workspace` (uint8 device tensor of
    :func:`das_workspace_bytes`) lets grids with few tiles or uneven work
    split each tile into items run by several workgroups; it is allocated
    when not given.  `plan` (a :class:`Plan` of this scan and record
    length) keeps the geometry tables in caller memory."""
    torch = _torch()
    lib = load()
    squeeze = rf.dim() == 3
    rf4 = rf.unsqueeze(0) if squeeze else rf
    if rf4.dim() != 4:
        raise ValueError("rf must be [F][T][C][S] or [T][C][S]")
    nf, nt, nc, ns = rf4.shape
    if nt != scan.n_tx or nc != scan.n_ch:
        raise ValueError(f"rf shape {tuple(rf.shape)} does not match n_tx={scan.n_tx}, "
                         f"n_ch={scan.n_ch}")
    g = scan.grid
    if out is None:
        out = torch.empty((nf, g.nz, g.nx), dtype=torch.float32, device=rf.device)
    elif out.dtype != torch.float32 or out.numel() != nf * g.nz * g.nx:
        raise ValueError("out must be float32 with F*nz*nx elements")
    if scan.mode not in ("stai", "pwi"):
        raise ValueError(f"mode must be 'stai' or 'pwi', got {scan.mode!r}")
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, nf, ns, _rf_dtype(rf4))
    rfp, outp, st = _dev(rf4, "rf"), _dev(out, "out"), _stream_ptr(rf4, stream)
    ph = _plan_arg(plan, scan, ns, rf.device)
    wsp, wsb, ws_keep = _workspace_arg(scan, ns, nf, workspace, rf.device, plan)
    if scan.mode == "stai":
        tx = keep.arr(ctypes.c_int32, scan.tx_elem)
        _lib.check(lib.wf_das_stai(rfp, probe, acq, tx, grid, ph, outp, wsp, wsb, st),
                   "wf_das_stai")
    else:
        ang = keep.arr(ctypes.c_double, scan.angles_rad)
        _lib.check(lib.wf_das_pwi(rfp, probe, acq, ang, _tref(scan), grid, ph, outp, wsp, wsb,
                                  st), "wf_das_pwi")
    del ws_keep  # the caching allocator keeps the block until the stream is done with it
    out = out.view(nf, g.nz, g.nx)
    return out[0] if squeeze else out


def das_noalloc(scan: Scan, rf, out=None, stream=None):
    """:func:`das` through ``wf_das_noalloc``: the library allocates no device
    memory for the call (its geometry tables and split partial frames live
    in a static per-GPU scratch array); overlapping calls on one GPU race."""
    torch = _torch()
    lib = load()
    squeeze = rf.dim() == 3
    rf4 = rf.unsqueeze(0) if squeeze else rf
    nf, nt, nc, ns = rf4.shape
    if nt != scan.n_tx or nc != scan.n_ch:
        raise ValueError(f"rf shape {tuple(rf.shape)} does not match n_tx={scan.n_tx}, "
                         f"n_ch={scan.n_ch}")
    g = scan.grid
    if out is None:
        out = torch.empty((nf, g.nz, g.nx), dtype=torch.float32, device=rf.device)
    elif out.dtype != torch.float32 or out.numel() != nf * g.nz * g.nx:
        raise ValueError("out must be float32 with F*nz*nx elements")
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, nf, ns, _rf_dtype(rf4))
    mode, tx, ang, tref = _mode_args(scan, keep)
    _lib.check(lib.wf_das_noalloc(mode, _dev(rf4, "rf"), probe, acq, tx, ang, tref, grid,
                                  _dev(out, "out"), _stream_ptr(rf4, stream)), "wf_das_noalloc")
    out = out.view(nf, g.nz, g.nx)
    return out[0] if squeeze else out


def das_stai(rf, scan: Scan, out=None, workspace=None, stream=None, plan=None):
    if scan.mode != "stai":
        raise ValueError("scan.mode must be 'stai'")
    return das(scan, rf, out=out, workspace=workspace, stream=stream, plan=plan)


def das_pwi(rf, scan: Scan, out=None, workspace=None, stream=None, plan=None):
    if scan.mode != "pwi":
        raise ValueError("scan.mode must be 'pwi'")
    return das(scan, rf, out=out, workspace=workspace, stream=stream, plan=plan)


TILE_INFO_FIELDS = ("px", "tile_z", "tile_x", "span", "nst", "slot", "lds_bytes", "ntz", "ntx",
                    "chunk", "threads", "nsplit", "split_chunks", "split_tx_parts",
                    "split_tx", "workgroups", "adjoint_threads", "adjoint_px",
                    "adjoint_tile_z", "adjoint_nsplit")


def tile_info(scan: Scan, n_s: int, n_frames: int = 1, dtype: int = 0) -> dict:
    """Launch plan of the DAS kernel for this geometry (host only, no GPU)."""
    lib = load()
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, n_frames, n_s, dtype)
    mode = 0 if scan.mode == "stai" else 1
    tx = keep.arr(ctypes.c_int32, scan.tx_elem) if mode == 0 else None
    ang = keep.arr(ctypes.c_double, scan.angles_rad) if mode == 1 else None
    tref = _tref(scan) if mode == 1 else 0
    info = (ctypes.c_int32 * len(TILE_INFO_FIELDS))()
    _lib.check(lib.wf_das_tile_info(mode, probe, acq, tx, ang, tref, grid,
                                    ctypes.cast(info, _lib.c_int32_p)), "wf_das_tile_info")
    return dict(zip(TILE_INFO_FIELDS, list(info)))


def delays(scan: Scan, device="cuda", stream=None):
    """Device-computed one-way delays in samples as float64 tensors:
    (tx [T][nz][nx] = (tau_tx - t0) fs, rx [C][nz][nx] = tau_rx fs)."""
    torch = _torch()
    lib = load()
    g = scan.grid
    mk = lambda n: torch.empty((n, g.nz, g.nx), dtype=torch.float32, device=device)
    txh, txl, rxh, rxl = mk(scan.n_tx), mk(scan.n_tx), mk(scan.n_ch), mk(scan.n_ch)
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep)
    mode = 0 if scan.mode == "stai" else 1
    tx = keep.arr(ctypes.c_int32, scan.tx_elem) if mode == 0 else None
    ang = keep.arr(ctypes.c_double, scan.angles_rad) if mode == 1 else None
    tref = _tref(scan) if mode == 1 else 0
    _lib.check(lib.wf_delays(mode, probe, acq, tx, ang, tref, grid, _dev(txh, "tx_hi"),
                             _dev(txl, "tx_lo"), _dev(rxh, "rx_hi"), _dev(rxl, "rx_lo"),
                             _stream_ptr(txh, stream)), "wf_delays")
    return (txh.double() + txl.double(), rxh.double() + rxl.double())


def envelope(bf, env=None, col_max=None, stream=None):
    """|analytic signal| along depth of bf [F][nz][nx] (or [nz][nx]);
    returns (env, col_max [F][nx])."""
    torch = _torch()
    lib = load()
    squeeze = bf.dim() == 2
    b3 = bf.unsqueeze(0) if squeeze else bf
    nf, nz, nx = b3.shape
    if env is None:
        env = torch.empty_like(b3)
    if col_max is None:
        col_max = torch.empty((nf, nx), dtype=torch.float32, device=bf.device)
    _lib.check(lib.wf_envelope(_dev(b3, "bf"), nf, nz, nx, _dev(env, "env"),
                               _dev(col_max, "col_max"), _stream_ptr(b3, stream)), "wf_envelope")
    env = env.view(nf, nz, nx)
    return (env[0] if squeeze else env), col_max


def log_compress(env, col_max, dr_db: float, offset: bool = False, out=None, stream=None):
    torch = _torch()
    lib = load()
    squeeze = env.dim() == 2
    e3 = env.unsqueeze(0) if squeeze else env
    nf, nz, nx = e3.shape
    if out is None:
        out = torch.empty_like(e3)
    flags = _lib.WF_BMODE_OFFSET if offset else 0
    _lib.check(lib.wf_log_compress(_dev(e3, "env"), _dev(col_max, "col_max"), nf, nz, nx,
                                   float(dr_db), flags, _dev(out, "out"),
                                   _stream_ptr(e3, stream)), "wf_log_compress")
    out = out.view(nf, nz, nx)
    return out[0] if squeeze else out


def bmode(bf, dr_db: float, offset: bool = False, out=None, col_max=None, stream=None):
    """Beamformed RF -> B-mode dB frame (envelope, frame max, 20 log10, clip)."""
    torch = _torch()
    lib = load()
    squeeze = bf.dim() == 2
    b3 = bf.unsqueeze(0) if squeeze else bf
    nf, nz, nx = b3.shape
    if out is None:
        out = torch.empty_like(b3)
    if col_max is None:
        col_max = torch.empty((nf, nx), dtype=torch.float32, device=bf.device)
    flags = _lib.WF_BMODE_OFFSET if offset else 0
    _lib.check(lib.wf_bmode(_dev(b3, "bf"), nf, nz, nx, float(dr_db), flags, _dev(out, "out"),
                            _dev(col_max, "col_max"), _stream_ptr(b3, stream)), "wf_bmode")
    out = out.view(nf, nz, nx)
    return out[0] if squeeze else out


# ---------------------------------------------------------------------------
# derivatives (adjoint w.r.t. RF, forward-mode d y / d c) and autograd
# ---------------------------------------------------------------------------

def fir(rf, taps: Sequence[float], out=None, stream=None):
    """FIR along the last (sample) axis of rf [..., S] (int16, float16 or
    float32), centred ('same' alignment, odd tap count <= 63); returns float32
    of rf's shape."""
    torch = _torch()
    lib = load()
    taps = [float(v) for v in taps]
    n_s = int(rf.shape[-1])
    n_rec = int(rf.numel() // n_s) if n_s else 0
    if out is None:
        out = torch.empty(rf.shape, dtype=torch.float32, device=rf.device)
    h = (ctypes.c_float * max(1, len(taps)))(*taps)
    _lib.check(lib.wf_fir(_dev(rf, "rf"), _rf_dtype(rf), n_rec, n_s, h, len(taps),
                          _dev(out, "out"), _stream_ptr(rf, stream)), "wf_fir")
    return out


def moments(env, wz: int, wx: int, sz: int, sx: int, out=None, stream=None):
    """Windowed moments of env [F][nz][nx] (or [nz][nx]): returns
    [F][3][mz][mx] (or [3][mz][mx]) holding E[X], E[X^2], E[X^3] of the
    wz x wx windows at origins (i sz, j sx)."""
    torch = _torch()
    lib = load()
    squeeze = env.dim() == 2
    e3 = env.unsqueeze(0) if squeeze else env
    nf, nz, nx = e3.shape
    if not (1 <= wz <= nz and 1 <= wx <= nx and sz >= 1 and sx >= 1):
        raise ValueError(f"window {wz}x{wx} / strides {sz},{sx} do not fit {nz}x{nx}")
    mz, mx = (nz - wz) // sz + 1, (nx - wx) // sx + 1
    if out is None:
        out = torch.empty((nf, 3, mz, mx), dtype=torch.float32, device=env.device)
    _lib.check(lib.wf_moments(_dev(e3, "env"), nf, nz, nx, int(wz), int(wx), int(sz), int(sx),
                              _dev(out, "out"), _stream_ptr(e3, stream)), "wf_moments")
    return out[0] if squeeze else out


def das_dydc(scan: Scan, rf, out=None, workspace=None, stream=None, plan=None):
    """d y / d c per pixel (forward mode), rf [F][T][C][S] -> [F][nz][nx]."""
    torch = _torch()
    lib = load()
    rf4 = rf.unsqueeze(0) if rf.dim() == 3 else rf
    nf, nt, nc, ns = rf4.shape
    g = scan.grid
    if out is None:
        out = torch.empty((nf, g.nz, g.nx), dtype=torch.float32, device=rf.device)
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, nf, ns, _rf_dtype(rf4))
    mode, tx, ang, tref = _mode_args(scan, keep)
    ph = _plan_arg(plan, scan, ns, rf.device)
    wsp, wsb, ws_keep = _workspace_arg(scan, ns, nf, workspace, rf.device, plan)
    _lib.check(lib.wf_das_dydc(mode, _dev(rf4, "rf"), probe, acq, tx, ang, tref, grid, ph,
                               _dev(out, "dydc"), wsp, wsb, _stream_ptr(rf4, stream)),
               "wf_das_dydc")
    del ws_keep
    return out


def adjoint_workspace_bytes(scan: Scan, n_s: int) -> int:
    """Device bytes of the workspace one :func:`das_adjoint` call needs."""
    lib = load()
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, 1, n_s, _lib.WF_RF_F32)
    mode, tx, ang, tref = _mode_args(scan, keep)
    n = ctypes.c_uint64(0)
    _lib.check(lib.wf_das_adjoint_workspace(mode, probe, acq, tx, ang, tref, grid,
                                            ctypes.byref(n)), "wf_das_adjoint_workspace")
    return int(n.value)


def das_adjoint(scan: Scan, g, n_s: int, out=None, workspace=None, stream=None, plan=None):
    """Adjoint of DAS: cotangent g [F][nz][nx] -> d L / d rf [F][T][C][S]
    (float32; per-tile fixed-point windows summed in tile order without
    global atomics, bitwise reproducible).  `workspace` (a uint8 device
    tensor of at least :func:`adjoint_workspace_bytes`) is allocated when
    not given."""
    torch = _torch()
    lib = load()
    g3 = g.unsqueeze(0) if g.dim() == 2 else g
    nf = g3.shape[0]
    if out is None:
        out = torch.empty((nf, scan.n_tx, scan.n_ch, n_s), dtype=torch.float32, device=g.device)
    ph = _plan_arg(plan, scan, n_s, g.device)
    if workspace is None:
        need = plan.workspace_bytes(1)[1] if plan is not None else adjoint_workspace_bytes(
            scan, n_s)
        workspace = torch.empty(need, dtype=torch.uint8, device=g.device)
    keep = _Keep()
    probe, acq, grid = _structs(scan, keep, nf, n_s, _lib.WF_RF_F32)
    mode, tx, ang, tref = _mode_args(scan, keep)
    _lib.check(lib.wf_das_adjoint(mode, probe, acq, tx, ang, tref, grid, ph, _dev(g3, "g"),
                                  _dev(out, "grad_rf"), _dev(workspace, "workspace"),
                                  ctypes.c_uint64(workspace.numel() * workspace.element_size()),
                                  _stream_ptr(g3, stream)),
               "wf_das_adjoint")
    return out


def dot(a, b, out=None, stream=None):
    """sum(a * b) of two float32 device tensors, deterministic."""
    torch = _torch()
    lib = load()
    if a.numel() != b.numel():
        raise ValueError("dot: size mismatch")
    if out is None:
        out = torch.empty((1,), dtype=torch.float32, device=a.device)
    _lib.check(lib.wf_dot(_dev(a, "a"), _dev(b, "b"), a.numel(), _dev(out, "out"),
                          _stream_ptr(a, stream)), "wf_dot")
    return out


def _autograd_function():
    torch = _torch()

    class DASFunction(torch.autograd.Function):
        """y = DAS(rf; c) with gradients w.r.t. the RF (adjoint kernel) and
        the speed of sound (forward-mode d y / d c reduced against dL/dy).
        ``c`` is a 0-dim tensor; its value is read on the host.  Each
        forward builds a :class:`Plan` for its c in torch-allocated device
        memory, so learning c adds nothing to the library's own cache."""

        @staticmethod
        def forward(ctx, rf, c, scan):
            scan_c = dataclasses.replace(scan, c=float(c))
            plan = Plan(scan_c, rf.shape[-1], device=rf.device)
            ctx.scan = scan_c
            ctx.plan = plan
            ctx.rf_dtype = rf.dtype
            ctx.save_for_backward(rf)
            return das(scan_c, rf, plan=plan)

        @staticmethod
        def backward(ctx, gy):
            (rf,) = ctx.saved_tensors
            gy = gy.contiguous().float()
            grad_rf = grad_c = None
            if ctx.needs_input_grad[0]:
                squeeze = rf.dim() == 3
                g3 = gy.unsqueeze(0) if squeeze else gy
                grad_rf = das_adjoint(ctx.scan, g3, rf.shape[-1],
                                      plan=ctx.plan).to(ctx.rf_dtype)
                grad_rf = grad_rf[0] if squeeze else grad_rf
            if ctx.needs_input_grad[1]:
                dydc = das_dydc(ctx.scan, rf, plan=ctx.plan)
                grad_c = dot(gy.reshape(-1), dydc.reshape(-1)).reshape(())
            return grad_rf, grad_c, None

    return DASFunction


_das_fn = None


def __getattr__(name):
    if name == "DASFunction":
        global _das_fn
        if _das_fn is None:
            _das_fn = _autograd_function()
        return _das_fn
    raise AttributeError(name)


def das_autograd(scan: Scan, rf, c):
    """Differentiable DAS: rf (float32/float16, requires_grad allowed) and the
    speed of sound c (0-dim tensor, requires_grad allowed)."""
    fn = __getattr__("DASFunction")
    return fn.apply(rf, c, scan)
