"""Builds librfd.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2302_00942_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "librfd.so")
BUILD = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function",
          # no packed-FP32 instructions anywhere in the device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the host sampler must evaluate float64 expressions exactly as written
HOST_EXTRA = {"host_plan.cpp": ["-ffp-contract=off"]}
SOURCES = ["k_stream.hip", "k_phi1.hip", "host_plan.cpp", "batch_server.cpp", "loop.cpp", "wide.cpp", "gw.cpp", "k_gw.hip", "spectrum.cpp", "k_spectrum.hip", "server.cpp", "autotune.cpp", "profile.cpp", "noalloc.hip", "bary.cpp", "k_bary.hip"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: install ROCm or put hipcc on PATH")
    return exe


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), *COMMON, *HOST_EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    # native driver of the C ABI (profiling runs), linked against librfd.so
    drv = os.path.join(HERE, "rfd_run")
    cmd = [hipcc(), "-O2", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, os.path.join(CSRC, "rfd_run.cpp"),
           "-L", HERE, "-lrfd", "-ldl", "-Wl,-rpath,$ORIGIN", "-o", drv + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(drv + ".tmp", drv)
    if verbose:
        print("built", OUT, "and", drv)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
