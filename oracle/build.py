"""Compile the CPU oracle (test infrastructure) into oracle/libsco.so.

Plain C11, -O2, no contraction of a*b+c into fused multiply-adds, no fast
math: every float operation is the IEEE-754 binary32 operation written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsco.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "sco.c")
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
