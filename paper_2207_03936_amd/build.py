"""Build the gfx950 shared library ``libsbt.so`` in-tree with hipcc.

Flags: whole-program compilation (one translation unit for the kernels, no
relocatable device code), -O3, -ffp-contract=off (binary32 expressions are
evaluated exactly as written, no fused multiply-add), no fast-math (division
stays correctly rounded, denormals are kept), and packed-FP32 instructions
disabled.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsbt.so")
SOURCES = [os.path.join(CSRC, "sbt.hip"), os.path.join(CSRC, "sbt_server.cpp")]
ARCH = os.environ.get("SBT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def command(out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-o", out] + SOURCES


def build(verbose: bool = False) -> str:
    """Compile ``libsbt.so`` (always recompiles) and return its path."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
