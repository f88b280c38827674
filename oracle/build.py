"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP for the thread pool over independent gates.  Fast-math is
off and floating-point contraction is disabled so that the Gaussian sampler
gives the same doubles as any other build of the same formula.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "locpir_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def sanitizer_runtime() -> str | None:
    """The shared address-sanitizer runtime of the ROCm clang, which both
    sanitizer builds link against (preload it into an unsanitized Python)."""
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def build_sanitized(outdir: str, verbose: bool = False) -> str:
    """The same oracle under the address and undefined-behaviour sanitizers
    (ROCm clang, shared sanitizer runtime, OpenMP from its libomp), into
    outdir/liboracle.so; load it with LOCPIR_ORACLE_LIB."""
    out = os.path.join(outdir, "liboracle.so")
    san = "-fsanitize=address,undefined -shared-libasan -fno-omit-frame-pointer".split()
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", *san, "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
