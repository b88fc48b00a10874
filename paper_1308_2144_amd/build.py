"""Compile libhb.so (HIP kernels for gfx950 + the C-ABI host code) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhb.so")
SOURCES = ["hb_kernels.hip", "hb_api.cpp", "hb_serve.cpp", "hb_tune.cpp", "hb_static.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the FP64 accumulators must round exactly as written.
# -packed-fp32-ops off: packed FP32 instructions are not used on this target.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-x", "hip",
]


def build(verbose: bool = False, out: str = LIB, defines: dict | None = None) -> str:
    """Compile the library to `out`; `defines` sets compile-time tuning macros
    (HB_U, HB_WAVES, HB_NT)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    dflags = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    cmd = [HIPCC] + FLAGS + dflags + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
