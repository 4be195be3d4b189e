"""Builds libbilu.so for gfx950 in-tree (paper_1703_01325_amd/_build/).

hipcc compiles the HIP translation unit for the device (gfx950) and the
host; g++ compiles the host-only analysis.  Every HIP compile carries
``-Xclang -target-feature -Xclang -packed-fp32-ops`` (no packed FP32 ops).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libbilu.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", f"-I{INC}", f"-I{CSRC}"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", f"-I{INC}", f"-I{CSRC}",
             f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    jobs = [
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "bilu_api.hip"),
         "-o", os.path.join(OUT_DIR, "bilu_api.o")],
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "analysis.cpp"),
         "-o", os.path.join(OUT_DIR, "analysis.o")],
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}",
          os.path.join(OUT_DIR, "bilu_api.o"), os.path.join(OUT_DIR, "analysis.o"),
          "-o", tmp, f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
