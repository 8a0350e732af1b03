"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/wf.h, and rejects bad arguments before any device call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(wf_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1811_01566_amd import _lib

    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wf_das_stai", "wf_das_pwi", "wf_envelope", "wf_bmode", "wf_log_compress",
              "wf_delays", "wf_last_error", "wf_abi_version", "wf_geometry_cache_clear",
              "wf_plan_bytes_stai", "wf_plan_bytes_pwi", "wf_plan_build_stai",
              "wf_plan_build_pwi", "wf_plan_destroy", "wf_plan_workspace",
              "wf_geometry_cache_info"):
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    from paper_1811_01566_amd import _lib

    for n in _declared():
        assert hasattr(lib, n), f"{n} declared in wf.h but not exported"
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"


def test_abi_version(lib):
    from paper_1811_01566_amd import _lib

    assert lib.wf_abi_version() == _lib.WF_ABI_VERSION == 8


def _geom(n_elem=8, n_tx=4, n_ch=8, n_s=256):
    from paper_1811_01566_amd import _lib

    probe = _lib.WfProbe(n_elem, 0.3e-3, None)
    acq = _lib.WfAcq(1, n_tx, n_ch, n_s, 0, 1540.0, 50e6, 0.0, 0.0, None)
    grid = _lib.WfGrid(16, 8, 5e-3, 0.1e-3, -1e-3, 0.2e-3)
    return probe, acq, grid


def _err(lib):
    return lib.wf_last_error().decode()


FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("field,value,code,needle", [
    ("n_tx", 0, -1, "n_tx"),
    ("n_ch", 2000, -1, "n_ch"),
    ("n_s", 100, -2, "multiple of 8"),
    ("c", -1.0, -1, "acq->c"),
    ("fs", 0.0, -1, "acq->fs"),
    ("f_number", -0.5, -1, "f_number"),
    ("dtype", 7, -1, "dtype"),
    ("n_frames", 0, -1, "n_frames"),
])
def test_acq_validation(lib, field, value, code, needle):
    probe, acq, grid = _geom()
    setattr(acq, field, value)
    st = lib.wf_das_stai(FAKE, probe, acq, None, grid, None, FAKE, None, 0, None)
    assert st == code
    assert needle in _err(lib)


def test_null_and_alignment_errors(lib):
    probe, acq, grid = _geom()
    assert lib.wf_das_stai(None, probe, acq, None, grid, None, FAKE, None, 0, None) == -1
    assert "rf is NULL" in _err(lib)
    assert lib.wf_das_stai(ctypes.c_void_p(0x10002), probe, acq, None, grid, None, FAKE, None, 0, None) == -2
    assert "16-byte" in _err(lib)
    assert lib.wf_das_stai(FAKE, None, acq, None, grid, None, FAKE, None, 0, None) == -1
    assert lib.wf_das_stai(FAKE, probe, acq, None, None, None, FAKE, None, 0, None) == -1


def test_transmit_and_angle_validation(lib):
    probe, acq, grid = _geom()
    bad = (ctypes.c_int32 * 4)(0, 1, 2, 9)
    assert lib.wf_das_stai(FAKE, probe, acq, bad, grid, None, FAKE, None, 0, None) == -1
    assert "tx_elem[3]" in _err(lib)
    ang = (ctypes.c_double * 4)(0.0, 0.1, 1.5, 0.0)
    assert lib.wf_das_pwi(FAKE, probe, acq, ang, 0, grid, None, FAKE, None, 0, None) == -1
    assert "angles_rad[2]" in _err(lib)
    ok = (ctypes.c_double * 4)(0.0, 0.1, 0.2, 0.0)
    assert lib.wf_das_pwi(FAKE, probe, acq, ok, 5, grid, None, FAKE, None, 0, None) == -1
    assert "tref" in _err(lib)
    assert lib.wf_das_pwi(FAKE, probe, acq, None, 0, grid, None, FAKE, None, 0, None) == -1


def test_channel_map_validation(lib):
    from paper_1811_01566_amd import _lib

    probe, acq, grid = _geom()
    rx = (ctypes.c_int32 * 8)(0, 1, 2, 3, 4, 5, 6, 8)
    acq.rx_elem = ctypes.cast(rx, _lib.c_int32_p)
    assert lib.wf_das_stai(FAKE, probe, acq, None, grid, None, FAKE, None, 0, None) == -1
    assert "rx_elem[7]" in _err(lib)


def test_overlap_rejected(lib):
    probe, acq, grid = _geom()
    assert lib.wf_das_stai(FAKE, probe, acq, None, grid, None, ctypes.c_void_p(0x10000 + 64), None, 0, None) == -1
    assert "overlaps" in _err(lib)


def test_image_call_validation(lib):
    assert lib.wf_envelope(FAKE, 1, 100, 4, ctypes.c_void_p(0x900000), ctypes.c_void_p(0xA00000), None) == -2
    assert "power of two" in _err(lib)
    assert lib.wf_envelope(None, 1, 128, 4, FAKE, FAKE, None) == -1
    assert lib.wf_log_compress(FAKE, ctypes.c_void_p(0x900000), 1, 8, 8, ctypes.c_float(0.0), 0,
                               FAKE, None) == -1
    assert "dr_db" in _err(lib)
    assert lib.wf_log_compress(FAKE, ctypes.c_void_p(0x900000), 1, 8, 8, ctypes.c_float(60.0), 4,
                               FAKE, None) == -1
    assert "flags" in _err(lib)
    assert lib.wf_bmode(FAKE, 1, 8, 8, ctypes.c_float(60.0), 0, FAKE, ctypes.c_void_p(0x900000),
                        None) == -1
    assert "overlaps" in _err(lib)
    assert lib.wf_delays(3, None, None, None, None, 0, None, FAKE, FAKE, FAKE, FAKE, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch

    import paper_1811_01566_amd as wf

    scan = wf.Scan(mode="pwi", n_elem=8, pitch=0.3e-3, c=1540.0, fs=50e6, n_tx=2, n_ch=8,
                   grid=wf.Grid(16, 8, 5e-3, 0.1e-3, -1e-3, 0.2e-3), angles_rad=(0.0, 0.1))
    rf = torch.zeros((2, 8, 256), dtype=torch.int16)
    with pytest.raises(ValueError, match="GPU"):
        wf.das(scan, rf)


def test_noalloc_checks_arguments_before_the_device(lib):
    """wf_das_noalloc validates like wf_das_pwi / wf_das_stai before it looks
    up its scratch or touches the device."""
    probe, acq, grid = _geom()
    ang = (ctypes.c_double * 4)(-0.1, 0.0, 0.05, 0.1)
    rf = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x8000000)
    assert lib.wf_das_noalloc(2, rf, probe, acq, None, ang, 0, grid, out, None) == -1
    assert "mode" in _err(lib)
    assert lib.wf_das_noalloc(1, None, probe, acq, None, ang, 0, grid, out, None) == -1
    assert "rf is NULL" in _err(lib)
    assert lib.wf_das_noalloc(1, rf, probe, acq, None, ang, 0, grid, None, None) == -1
    assert "out is NULL" in _err(lib)
    assert lib.wf_das_noalloc(1, rf, probe, acq, None, None, 0, grid, out, None) == -1
    acq.n_s = 250
    assert lib.wf_das_noalloc(0, rf, probe, acq, None, None, 0, grid, out, None) == -2
    assert "multiple of 8" in _err(lib)
