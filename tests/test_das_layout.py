"""The LDS layout of the DAS kernels (CPU): the host-compiled layout check,
and the LDS the launch plan reports against that layout."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_01566_amd", "csrc")


def _cxx():
    for c in (os.environ.get("CXX"), "g++", "c++", "clang++"):
        if c and shutil.which(c):
            return shutil.which(c)
    pytest.skip("no host C++ compiler")


def test_layout_check_program(tmp_path):
    exe = tmp_path / "das_layout_check"
    src = os.path.join(ROOT, "tests", "das_layout_check.cpp")
    subprocess.run([_cxx(), "-std=c++17", "-O1", "-Wall", f"-I{CSRC}", src, "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout


def _layout_total(nbuf, slot, T, chunk=16):
    return nbuf * chunk * slot * 8 + 32 * T + chunk * 2 * 4


@pytest.mark.parametrize("name,dtype,pp", [("pwi", 0, 2), ("pwi", 2, 1), ("stai_full", 0, 1),
                                           ("stai_small", 0, 1)])
def test_reported_lds_matches_layout(name, dtype, pp):
    """tile_info's LDS per workgroup is the layout of 2 window buffers per
    pass staged per barrier: two passes for 16-bit RF on 1024-thread tiles
    where they fit, one otherwise (FP32 RF, smaller tiles)."""
    import phantom
    from wfhelp import scan_from_workload

    import paper_1811_01566_amd as wf

    w = phantom.get_workload(name)
    info = wf.tile_info(scan_from_workload(w), w.n_s, 1, dtype)
    assert info["lds_bytes"] == _layout_total(2 * pp, info["slot"], w.n_tx)
    assert info["lds_bytes"] <= 163840
    if pp == 2:
        assert info["threads"] == 1024
