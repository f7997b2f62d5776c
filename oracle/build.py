"""Build the CPU oracle (test infrastructure) as oracle/liboracle.so.

Compiled with gcc, -ffp-contract=off and no fast-math, so the binary32
decisions follow the stated formula operation by operation (SSE arithmetic,
correctly rounded division, fmaf from libm, rintf ties-to-even).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "adop_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-msse2", "-mfpmath=sse", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
