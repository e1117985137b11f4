"""Compiles the HIP library in-tree: paper_1411_5373_amd/libfdmt.so (gfx950).

The table builder is plain C++ compiled by g++ with FP contraction off (its
float64 arithmetic must be evaluated exactly as written); kernels and the C
ABI are HIP compiled by hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfdmt.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
CXX_FLAGS = ["-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]

HIP_SOURCES = ["fdmt_kernels.hip", "fdmt_gather.hip", "fdmt_narrow.hip", "fdmt_adjoint.hip", "fdmt_boxcar.hip",
               "fdmt_fft.hip", "fdmt_copy.hip", "fdmt_api.hip"]
LIBS = ["-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib",  # FFT-FDMT's transforms
        "-ldl"]  # dladdr: the tuning cache beside the library
CXX_SOURCES = ["fdmt_tables.cpp", "fdmt_schedule.cpp", "fdmt_tune.cpp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libfdmt.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
            for src in CXX_SOURCES]
    jobs += [([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
             for src in HIP_SOURCES]
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as pool:
        list(pool.map(lambda cmd: _run(cmd, verbose), jobs))
    objs = [cmd[-1] for cmd in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    print(build(verbose=True))
