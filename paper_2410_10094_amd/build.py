"""Builds the HIP library ``libsptc.so`` for gfx950 with hipcc.

    python -m paper_2410_10094_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libsptc.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "grouped.hip"), os.path.join(CSRC, "batch.hip"),
           os.path.join(CSRC, "block_mfma.hip"), os.path.join(CSRC, "queue.hip"), os.path.join(CSRC, "xpart.hip"), os.path.join(CSRC, "noalloc.hip"), os.path.join(CSRC, "sptc.cpp")]
HEADERS = [os.path.join(CSRC, "sptc_internal.hpp"), os.path.join(CSRC, "prim.hpp"), os.path.join(CSRC, "xpart.hpp"), os.path.join(ROOT, "include", "sptc.h")]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-function",
    # hardware FP64 atomic add instead of a CAS loop
    "-munsafe-fp-atomics",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA operands and accumulators in VGPRs: without it the FP64 MFMA
    # accumulators are copied between AGPRs and VGPRs around every step
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-fvisibility=hidden",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source into libsptc.so (always recompiles)."""
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
