"""Builds libgsr.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsr.so")
SOURCES = [os.path.join(CSRC, "gsr_api.cpp"), os.path.join(CSRC, "gsr_kernels.hip"),
           os.path.join(CSRC, "gsr_raster.hip"), os.path.join(CSRC, "gsr_optim.hip"),
           os.path.join(CSRC, "gsr_fcs.hip"), os.path.join(CSRC, "gsr_partition.cpp"),
           os.path.join(CSRC, "gsr_densify.hip"), os.path.join(CSRC, "gsr_static.hip")]
HEADERS = [os.path.join(ROOT, "include", "gsr.h"), os.path.join(CSRC, "gsr_internal.h"),
           os.path.join(CSRC, "gsr_device.h"), os.path.join(CSRC, "gsr_stages.h"),
           os.path.join(CSRC, "gsr_cull.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # identical float32 expressions in the forward and reverse kernels
    "-ffp-contract=off",
    # no packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_2510_01767_amd/libgsr.so."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
