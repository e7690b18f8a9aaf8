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
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("SBT_OFFLOAD_ARCH", "gfx950")
# persistent kernels: one translation unit per workgroup width, built in parallel
WIDTHS = (64, 128, 256, 512, 1024)


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def compile_commands() -> list:
    """(object path, hipcc command) for every translation unit."""
    inc = ["-I", INCLUDE, "-I", CSRC]
    out = []
    for name in ("sbt", "sbt_server"):
        src = os.path.join(CSRC, name + (".hip" if name == "sbt" else ".cpp"))
        obj = os.path.join(OBJDIR, name + ".o")
        out.append((obj, [hipcc()] + FLAGS + inc + ["-c", src, "-o", obj]))
    for b in WIDTHS:
        obj = os.path.join(OBJDIR, f"sbt_persistent_{b}.o")
        out.append((obj, [hipcc()] + FLAGS + inc + [f"-DSBT_TPE={b}", "-c",
                                                    os.path.join(CSRC, "sbt_persistent.hip"), "-o", obj]))
    return out


def command(out: str = LIB) -> list:
    """Link command of the shared library from the objects."""
    return [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", out] + [o for o, _ in compile_commands()]


def build(verbose: bool = False) -> str:
    """Compile ``libsbt.so`` (always recompiles) and return its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = compile_commands()
    procs = []
    for obj, cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    errors = []
    for p in procs:
        so, se = p.communicate()
        if p.returncode != 0:
            errors.append(so + se)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
