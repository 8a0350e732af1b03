"""ctypes declarations of libwf.so (the C ABI in include/wf.h)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwf.so")

WF_OK = 0
WF_ERR_INVALID_ARG = -1
WF_ERR_UNSUPPORTED = -2
WF_ERR_DEVICE = -3
WF_ERR_WORKSPACE = -4
WF_ABI_VERSION = 8
WF_PLAN_DELAY_TABLES = 1  # plan flag: window-local delay tables in the plan

WF_RF_I16, WF_RF_F16, WF_RF_F32 = 0, 1, 2
WF_PWI_TREF_FIRST, WF_PWI_TREF_CENTRE = 0, 1
WF_BMODE_OFFSET = 1

c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_double_p = ctypes.POINTER(ctypes.c_double)
c_float_p = ctypes.c_void_p  # device pointers are passed as integers


class WfProbe(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("pitch", ctypes.c_double), ("elem_x", c_double_p)]


class WfGrid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("z0", ctypes.c_double),
                ("dz", ctypes.c_double), ("x0", ctypes.c_double), ("dx", ctypes.c_double)]


class WfAcq(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("n_tx", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("n_s", ctypes.c_int32), ("dtype", ctypes.c_int32), ("c", ctypes.c_double),
                ("fs", ctypes.c_double), ("t0", ctypes.c_double), ("f_number", ctypes.c_double),
                ("rx_elem", c_int32_p)]


P = ctypes.POINTER
V = ctypes.c_void_p
I = ctypes.c_int32
F = ctypes.c_float

# name -> (restype, argtypes); every function declared in include/wf.h
SIGNATURES = {
    "wf_das_stai": (I, [V, P(WfProbe), P(WfAcq), c_int32_p, P(WfGrid), V, V, V,
                        ctypes.c_uint64, V]),
    "wf_das_pwi": (I, [V, P(WfProbe), P(WfAcq), c_double_p, I, P(WfGrid), V, V, V,
                       ctypes.c_uint64, V]),
    "wf_das_workspace": (I, [I, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid),
                             ctypes.POINTER(ctypes.c_uint64)]),
    "wf_delays": (I, [I, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid), V, V, V, V,
                      V]),
    "wf_das_tile_info": (I, [I, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid),
                             c_int32_p]),
    "wf_das_dydc": (I, [I, V, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid), V, V,
                        V, ctypes.c_uint64, V]),
    "wf_das_noalloc": (I, [I, V, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid), V,
                           V]),
    "wf_das_adjoint": (I, [I, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I, P(WfGrid), V, V,
                           V, V, ctypes.c_uint64, V]),
    "wf_plan_bytes_stai": (I, [P(WfProbe), P(WfAcq), c_int32_p, P(WfGrid), I,
                               ctypes.POINTER(ctypes.c_uint64)]),
    "wf_plan_bytes_pwi": (I, [P(WfProbe), P(WfAcq), c_double_p, I, P(WfGrid), I,
                              ctypes.POINTER(ctypes.c_uint64)]),
    "wf_plan_build_stai": (I, [P(WfProbe), P(WfAcq), c_int32_p, P(WfGrid), I, V,
                               ctypes.c_uint64, ctypes.POINTER(V), V]),
    "wf_plan_build_pwi": (I, [P(WfProbe), P(WfAcq), c_double_p, I, P(WfGrid), I, V,
                              ctypes.c_uint64, ctypes.POINTER(V), V]),
    "wf_plan_destroy": (None, [V]),
    "wf_plan_workspace": (I, [V, I, ctypes.POINTER(ctypes.c_uint64),
                              ctypes.POINTER(ctypes.c_uint64)]),
    "wf_geometry_cache_info": (I, [ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "wf_das_adjoint_workspace": (I, [I, P(WfProbe), P(WfAcq), c_int32_p, c_double_p, I,
                                     P(WfGrid), ctypes.POINTER(ctypes.c_uint64)]),
    "wf_dot": (I, [V, V, ctypes.c_int64, V, V]),
    "wf_envelope": (I, [V, I, I, I, V, V, V]),
    "wf_log_compress": (I, [V, V, I, I, I, F, I, V, V]),
    "wf_bmode": (I, [V, I, I, I, F, I, V, V, V]),
    "wf_fir": (I, [V, I, ctypes.c_int64, I, ctypes.POINTER(ctypes.c_float), I, V, V]),
    "wf_moments": (I, [V, I, I, I, I, I, I, I, V, V]),
    "wf_last_error": (ctypes.c_char_p, []),
    "wf_abi_version": (I, []),
    "wf_geometry_cache_clear": (I, []),
}

_lib = None


class WfError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} failed ({status}): {msg}")
        self.status = status


def load(path: str = None) -> ctypes.CDLL:
    """Load libwf.so (or the library named by $WF_LIB); raises if it has not
    been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("WF_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1811_01566_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, fn: str) -> None:
    if status != WF_OK:
        msg = _lib.wf_last_error().decode("utf-8", "replace") if _lib else ""
        raise WfError(status, fn, msg)
