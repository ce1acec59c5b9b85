"""Build the MOFF HIP library for gfx950 (in-tree: paper_1510_08318_amd/libmoff.so).

    python -m paper_1510_08318_amd.build      (or __graft_entry__.build())

The host plan (plan.cpp) is compiled by g++ without floating-point contraction so
that footprint cells follow their IEEE double definition exactly; the HIP
sources are compiled by hipcc for gfx950 with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmoff.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}):\n{' '.join(cmd)}\n{r.stdout}")
    return r.stdout


def build(verbose: bool = False, extra_hip_flags=None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]
    jobs = []
    gxx = shutil.which("g++") or "g++"
    objs = []
    for src in ("plan.cpp", "fx_tables.cpp"):
        o = os.path.join(BUILD, src.replace(".cpp", ".o"))
        jobs.append([gxx, *HOST_FLAGS, *inc, "-I", os.path.join(ROCM, "include"), "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in ("kernels.hip", "mfma.hip", "uv_autocorr.hip", "fx.hip", "capi.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        jobs.append([HIPCC, *HIP_FLAGS, *(extra_hip_flags or []), *inc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=7) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
