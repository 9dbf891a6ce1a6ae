"""Compile the HIP/C++ sources of the operator library into libwf.so (gfx950).

Usage: python paper_2605_26347_amd/build_lib.py   (by path: importing the package would
load the library it builds), or __graft_entry__.build().
Each translation unit is compiled by hipcc in parallel, then linked as one shared
library next to this file.  FP32 packed-math instructions are disabled for all device
code; the FP64 build kernels are compiled without floating-point contraction so that
their integer decisions (bins, cells, kernel sides, thresholds) are reproducible.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libwf.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("WF_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "k_fft.hip": [],
    "k_grid.hip": [],
    "k_build.hip": ["-ffp-contract=off"],
    "k_util.hip": [],
    "k_mlp.hip": [],
    "k_holo.hip": [],
    "k_weight.hip": ["-ffp-contract=off"],
    "wf_weight.cpp": [],
    "wf_mlp.cpp": [],
    "host_plan.cpp": ["-ffp-contract=off"],
    "wf_abi.cpp": [],
}


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _common():
    return [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc()] + _common() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        futs = {ex.submit(_compile, s, e): s for s, e in SOURCES.items()}
        objs = [f.result() for f in futs]
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    return OUT


# Host-side AddressSanitizer build (CPU checks of the host C++: planner, partitioning,
# argument paths).  Only host code is instrumented (each sanitizer flag is scoped to the
# host pass); the device objects of the regular build are linked unchanged.
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_OUT = os.path.join(ASAN_DIR, "libwf_asan.so")
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the sanitizer runtime the instrumented library needs preloaded."""
    clang = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "llvm", "bin",
                         "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    return r.stdout.strip()


def build_asan(verbose: bool = True) -> str:
    os.makedirs(ASAN_DIR, exist_ok=True)
    dev = [os.path.join(BUILD, s + ".o") for s in SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev):
        build(verbose)

    def host(src):
        obj = os.path.join(ASAN_DIR, src + ".o")
        cmd = ([_hipcc()] + _common() + SOURCES[src] + ASAN_HOST + ["-g", "-O1", "-c",
               os.path.join(CSRC, src), "-o", obj])
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(host, HOST_SOURCES))
    cmd = ([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host",
            "-fsanitize=address", "-Xarch_host", "-shared-libasan", "-o", ASAN_OUT]
           + objs + dev)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    if verbose:
        print(f"built {ASAN_OUT}", file=sys.stderr)
    return ASAN_OUT


if __name__ == "__main__":
    if "--asan" in sys.argv:
        build_asan()
    else:
        build()
