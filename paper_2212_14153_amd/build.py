"""Build the HIP library ``libfpdlbm.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfpdlbm.so")
SOURCES = ["fpd_kernels.hip", "fpd_runtime.hip"]
ARCH = os.environ.get("FPD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: scalar and float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FMA only where one source expression is a*b+c: rounding then does not depend on
    # how a template instance is unrolled or scheduled (bitwise-stable launch shapes)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


# roctx ranges around the C ABI calls (rocprofv3 --marker-trace)
LIBS = ["-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES], *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
