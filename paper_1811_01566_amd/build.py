"""Compile libwf.so (HIP for gfx950) in-tree.

    python -m paper_1811_01566_amd.build             # libwf.so
    python -m paper_1811_01566_amd.build --sanitize  # libwf_asan.so

Packed FP32 instructions are disabled for device code
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host pass warns
that it does not know the feature, which is harmless.

``--sanitize`` builds the host library (argument checks, launch and split
planning, plans and the geometry cache in ``api.cpp``) with the host
compiler under AddressSanitizer and UndefinedBehaviorSanitizer, and links it
with the kernels built as usual (no sanitizer in device code).  Load it
through ``WF_LIB`` with the sanitizer runtimes preloaded, e.g.

    LD_PRELOAD="$(g++ -print-file-name=libasan.so) $(g++ -print-file-name=libubsan.so)" \
    ASAN_OPTIONS=detect_leaks=0 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    WF_LIB=paper_1811_01566_amd/libwf_asan.so python -m pytest tests -m "not gpu" -k \
        "abi or tile_plan or plan_cpu or das_layout"
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwf.so")
SOURCES = ["api.cpp", "das.hip", "adjoint.hip", "envelope.hip", "prefilter.hip", "noalloc.hip"]
ARCH = os.environ.get("WF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libwf.so)")


def compile_cmd(out: str) -> list:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-command-line-argument",
        f"-I{os.path.join(ROOT, 'include')}",
        "-o", out,
    ] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Every source compiled to an object in parallel (each carries its own
    device code; no kernel calls across files), then one shared link."""
    import tempfile

    flags = compile_cmd("unused")
    cc, opts = flags[0], [f for f in flags[1:] if f not in ("-shared", "-o", "unused")
                          and not f.endswith((".cpp", ".hip"))]
    opts += [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory() as tmpd:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src + ".o")
            objs.append(obj)
            cmd = [cc, *opts, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                          text=True))
        for p in procs:
            log = p.communicate()[0]
            if p.returncode != 0:
                sys.stderr.write(log)
                raise RuntimeError(f"hipcc failed with status {p.returncode}: {' '.join(p.args)}")
        tmp = out + f".tmp{os.getpid()}"
        link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc link failed with status {r.returncode}")
        os.replace(tmp, out)
    return out


LIB_ASAN = os.path.join(HERE, "libwf_asan.so")
HOST_SOURCES = ["api.cpp"]


def build_sanitized(verbose: bool = False, out: str = LIB_ASAN) -> str:
    """libwf with the host code under ASan + UBSan (see the module doc)."""
    import tempfile

    cxx = os.environ.get("CXX") or shutil.which("g++")
    if not cxx:
        raise RuntimeError("no host C++ compiler for the sanitized build")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    inc = f"-I{os.path.join(ROOT, 'include')}"
    with tempfile.TemporaryDirectory() as tmp:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            if src in HOST_SOURCES:
                cmds.append([cxx, "-std=c++17", "-O1", "-g", "-fPIC", "-Wall", *san,
                             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", inc, "-c",
                             os.path.join(CSRC, src), "-o", obj])
            else:
                cmds.append([hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
                             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                             "-Wno-unused-command-line-argument", inc, "-c",
                             os.path.join(CSRC, src), "-o", obj])
        procs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                          text=True))
        for p in procs:
            log = p.communicate()[0]
            if p.returncode != 0:
                sys.stderr.write(log)
                raise RuntimeError(f"compile failed: {' '.join(p.args)}")
        link = [cxx, "-shared", *san, "-o", out + ".tmp", *objs, "-L/opt/rocm/lib",
                "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link failed")
        os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        print(build_sanitized(verbose=True))
    else:
        print(build(verbose=True))
