"""Plans on the CPU (no GPU): sizes, argument checks that run before any
device call, and that sizing plans adds nothing to the library's own cache.

The geometry of a DAS call - probe, transmit sequence, speed of sound,
sampling rate and pixel grid (the metadata of Sec. II-A) - fixes its delay
tables and launch plan; a plan holds them in caller memory."""

import ctypes
import math

import numpy as np
import pytest

from paper_1811_01566_amd import _lib

FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: the checks fail first


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _pwi(c=1540.0, n_tx=16, n_ch=64, n_s=2048):
    probe = _lib.WfProbe(n_ch, 0.3e-3, None)
    acq = _lib.WfAcq(1, n_tx, n_ch, n_s, 0, c, 50e6, 0.0, 0.0, None)
    grid = _lib.WfGrid(256, 128, 5e-3, 25e-3 / 255, -9.45e-3, 18.9e-3 / 127)
    ang = (ctypes.c_double * n_tx)(*np.radians(np.linspace(-16, 16, n_tx)))
    return probe, acq, grid, ang


def _stai(c=1540.0, n=32, n_s=1024):
    probe = _lib.WfProbe(n, 0.3e-3, None)
    acq = _lib.WfAcq(1, n, n, n_s, 0, c, 50e6, 0.0, 0.0, None)
    grid = _lib.WfGrid(128, 128, 0.0, 30e-3 / 127, -4.65e-3, 9.3e-3 / 127)
    return probe, acq, grid


def _pwi_bytes(lib, probe, acq, grid, ang, flags=0):
    n = ctypes.c_uint64(0)
    st = lib.wf_plan_bytes_pwi(probe, acq, ang, 0, grid, flags, ctypes.byref(n))
    assert st == 0, lib.wf_last_error()
    return n.value


def _cache(lib):
    n, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
    assert lib.wf_geometry_cache_info(ctypes.byref(n), ctypes.byref(b)) == 0
    return n.value, b.value


def test_plan_bytes_hold_the_tables(lib):
    probe, acq, grid, ang = _pwi()
    b = _pwi_bytes(lib, probe, acq, grid, ang)
    # per-transmit (32 B) and per-channel (16 B) constants, each part aligned
    # to 256 bytes, then at least one word of work list
    tx = math.ceil(acq.n_tx * 32 / 256) * 256
    ch = math.ceil(acq.n_ch * 16 / 256) * 256
    assert b >= tx + ch + 256 and b % 256 == 0
    p, a, g = _stai()
    n = ctypes.c_uint64(0)
    assert lib.wf_plan_bytes_stai(p, a, None, g, 0, ctypes.byref(n)) == 0
    assert n.value >= math.ceil(32 * 32 / 256) * 256 + math.ceil(32 * 16 / 256) * 256


def _tile_slots(w):
    """Pixel slots of the launch plan: tiles x threads x pixels per thread."""
    import paper_1811_01566_amd as wf
    from wfhelp import scan_from_workload

    info = wf.tile_info(scan_from_workload(w), w.n_s, 1)
    return info["ntz"] * info["ntx"] * info["threads"] * info["px"]


@pytest.mark.parametrize("name", ["stai_small", "pwi", "paper_pwi"])
def test_delay_tables_add_one_word_per_slot_and_element(lib, name):
    """WF_PLAN_DELAY_TABLES adds, 256-byte aligned, 4 bytes per (pixel slot,
    channel padded to 16) and per (pixel slot, transmit), the latter for
    every tile shape but PWI on 1024 x 2 tiles."""
    import paper_1811_01566_amd as wf
    import phantom
    from wfhelp import scan_from_workload

    w = phantom.get_workload(name)
    scan = scan_from_workload(w)
    plain = wf.plan_bytes(scan, w.n_s, delay_tables=False)
    full = wf.plan_bytes(scan, w.n_s, delay_tables=True)
    slots = _tile_slots(w)
    rx = slots * math.ceil(w.n_ch / 16) * 16 * 4
    info = wf.tile_info(scan, w.n_s, 1)
    # transmit words for every tile shape but PWI on 1024 x 2 tiles
    pwi_large = w.mode == "pwi" and info["threads"] == 1024 and info["px"] == 2
    tx = 0 if pwi_large else slots * w.n_tx * 4
    align = lambda v: math.ceil(v / 256) * 256  # noqa: E731
    assert full - plain == align(rx) + align(tx)
    if name == "pwi":  # 1024 x 512 grid on 1024 x 2 tiles, 128 channels: 256 MiB
        assert pwi_large and full - plain == 256 << 20


def test_unknown_plan_flags_are_refused(lib):
    probe, acq, grid, ang = _pwi()
    n = ctypes.c_uint64(0)
    assert lib.wf_plan_bytes_pwi(probe, acq, ang, 0, grid, 2, ctypes.byref(n)) == -1
    assert "flags" in lib.wf_last_error().decode()
    out = ctypes.c_void_p(0x1)
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0x100, FAKE, 1 << 30,
                                 ctypes.byref(out), None) == -1
    assert out.value is None


def test_hundred_speeds_of_sound_add_nothing_to_the_cache(lib):
    """Learning c builds a plan per value: sizing and planning 100 distinct
    speeds of sound must leave the library's cache (host plans and device
    tables of plan-less calls) untouched."""
    before = _cache(lib)
    sizes = set()
    for c in np.linspace(1480.0, 1600.0, 100):
        probe, acq, grid, ang = _pwi(c=float(c))
        sizes.add(_pwi_bytes(lib, probe, acq, grid, ang))
    assert _cache(lib) == before
    assert len(sizes) >= 1


def test_plan_build_checks_before_the_device(lib):
    probe, acq, grid, ang = _pwi()
    need = _pwi_bytes(lib, probe, acq, grid, ang)
    out = ctypes.c_void_p(0x1)
    # no out pointer
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0, FAKE, need, None, None) == -1
    # no device memory
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0, None, need, ctypes.byref(out),
                                 None) == -1
    assert out.value is None  # cleared on failure
    # misaligned device memory
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0, ctypes.c_void_p(0x10040), need,
                                 ctypes.byref(out), None) == -1
    assert "256-byte" in lib.wf_last_error().decode()
    # too small: WF_ERR_WORKSPACE, nothing written
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0, FAKE, need - 256,
                                 ctypes.byref(out), None) == -4
    assert "needed" in lib.wf_last_error().decode()
    # an invalid geometry fails validation first
    acq.c = -1.0
    assert lib.wf_plan_build_pwi(probe, acq, ang, 0, grid, 0, FAKE, need, ctypes.byref(out),
                                 None) == -1
    p, a, g = _stai()
    a.n_tx = 0
    assert lib.wf_plan_build_stai(p, a, None, g, 0, FAKE, 1 << 20, ctypes.byref(out),
                                  None) == -1


def test_plan_destroy_and_queries_tolerate_null(lib):
    lib.wf_plan_destroy(None)
    d, a = ctypes.c_uint64(0), ctypes.c_uint64(0)
    assert lib.wf_plan_workspace(None, 1, ctypes.byref(d), ctypes.byref(a)) == -1
    assert lib.wf_geometry_cache_info(None, None) == -1


def test_binding_plan_bytes_match_the_library():
    import paper_1811_01566_amd as wf

    scan = wf.Scan(mode="pwi", n_elem=64, pitch=0.3e-3, c=1540.0, fs=50e6, n_tx=16, n_ch=64,
                   grid=wf.Grid(256, 128, 5e-3, 25e-3 / 255, -9.45e-3, 18.9e-3 / 127),
                   angles_rad=tuple(np.radians(np.linspace(-16, 16, 16))))
    probe, acq, grid, ang = _pwi()
    assert wf.plan_bytes(scan, 2048, delay_tables=False) == _pwi_bytes(_lib.load(), probe, acq,
                                                                       grid, ang)
    assert wf.plan_bytes(scan, 2048) == _pwi_bytes(_lib.load(), probe, acq, grid, ang,
                                                   _lib.WF_PLAN_DELAY_TABLES)


def test_binding_refuses_lists_shorter_than_the_geometry():
    """The library reads n_tx angles or transmit elements and n_ch channel
    elements from host arrays: the binding refuses shorter lists instead of
    letting the library read past them (a 6-transmit scan with 3 angles once
    gave a different plan key on every call)."""
    import paper_1811_01566_amd as wf
    import phantom

    grid = wf.Grid(64, 32, 5e-3, 1e-4, -4e-3, 2.5e-4)
    pwi = wf.Scan(mode="pwi", n_elem=32, pitch=0.3e-3, c=1540.0, fs=50e6, n_tx=6, n_ch=32,
                  grid=grid, angles_rad=(-0.2, 0.0, 0.15))
    with pytest.raises(ValueError, match="angles_rad has 3 entries, 6 expected"):
        wf.plan_bytes(pwi, 1024)
    stai = wf.Scan(mode="stai", n_elem=32, pitch=0.3e-3, c=1540.0, fs=50e6, n_tx=4, n_ch=32,
                   grid=grid, tx_elem=(0, 1, 2), rx_elem=tuple(range(32)))
    with pytest.raises(ValueError, match="tx_elem has 3 entries"):
        wf.das_workspace_bytes(stai, 1024)
    with pytest.raises(ValueError, match="rx_elem"):
        wf.plan_bytes(wf.Scan(mode="stai", n_elem=32, pitch=0.3e-3, c=1540.0, fs=50e6, n_tx=4,
                              n_ch=32, grid=grid, rx_elem=tuple(range(31))), 1024)
    with pytest.raises(ValueError, match="plane waves need as many angles_deg"):
        phantom.tiny_pwi(n_tx=6)
