"""Builds libbilu.so for gfx950 in-tree (paper_1703_01325_amd/_build/).

hipcc compiles the HIP translation units for the device (gfx950) and the
host -- the ABI and the non-sweep kernels (bilu_api.hip), the sweep and
SpMV kernels once per block size (sweep_b.hip with -DBILU_B=1..8), the
batch sweep (batch_sweep.hip) and the device symbolic phase (symbolic.hip)
-- in parallel; g++ compiles the host-only
analysis.  Every HIP compile carries
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
    objs = []
    jobs = []

    def hip_job(src, obj, *defs):
        objs.append(os.path.join(OUT_DIR, obj))
        jobs.append([hipcc, *HIP_FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", objs[-1]])

    hip_job("bilu_api.hip", "bilu_api.o")
    for b in range(1, 9):
        hip_job("sweep_b.hip", f"sweep_b{b}.o", f"-DBILU_B={b}")
    hip_job("batch_sweep.hip", "batch_sweep.o")
    hip_job("symbolic.hip", "symbolic.o")
    objs.append(os.path.join(OUT_DIR, "analysis.o"))
    jobs.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "analysis.cpp"), "-o", objs[-1]])
    workers = max(1, min(len(jobs), int(os.environ.get("BILU_BUILD_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
