"""Compile the HIP sources of the library into ``libadaptgrav.so`` (gfx950).

Every translation unit is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled; ``k_step.hip`` additionally disables fused
multiply-add contraction, because the timestep bin and the predictor are
defined one rounding per operation.  Objects go to ``_build/`` at the repo
root; the shared library is written next to this file.  ``peak/fma_peak`` is
the FMA issue-rate microbenchmark behind the VALU rooflines.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libadaptgrav.so")
PEAK_SRC = os.path.join(HERE, "peak", "fma_peak.hip")
PEAK_EXE = os.path.join(HERE, "peak", "fma_peak")

SOURCES = ["ag_api.hip", "k_direct.hip", "k_step.hip", "k_tree.hip", "k_walk.hip"]
EXTRA = {"k_step.hip": ["-ffp-contract=off"]}

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str) -> str:
    out = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return out


def build(verbose: bool = False) -> str:
    """Compile all sources (always; no staleness check) and link the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    # the VALU issue-rate microbenchmark (same code-generation flags)
    cmd = [HIPCC, *FLAGS, PEAK_SRC, "-o", PEAK_EXE + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for fma_peak.hip:\n{res.stderr}")
    os.replace(PEAK_EXE + ".tmp", PEAK_EXE)
    if verbose:
        print("built", LIB, "and", PEAK_EXE)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
