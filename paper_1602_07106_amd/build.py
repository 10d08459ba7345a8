"""Build libba.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1602_07106_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "ba.hip")
DEPS = [SRC, os.path.join(ROOT, "include", "ba.h")] + sorted(glob.glob(os.path.join(PKG, "csrc", "*.h")))
LIB = os.path.join(PKG, "libba.so")
# issue-rate and store-rate microbenchmarks that price the ALU roofline (bench.py --workload rates)
RATES_SRC = os.path.join(PKG, "csrc", "ba_rates.hip")
RATES_LIB = os.path.join(PKG, "libba_rates.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep hipcc from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str, lib: str, verbose: bool) -> None:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-o", tmp, src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compile libba.so and libba_rates.so; always recompiles (the build check
    must compile)."""
    _compile(SRC, LIB, verbose)
    _compile(RATES_SRC, RATES_LIB, verbose)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
