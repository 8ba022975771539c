"""Build the CPU oracle (plain C, gcc) into oracle/liboracle.so.

The oracle is test infrastructure: it is compiled so that the tests, the smoke
check and the benchmark's CPU-baseline leg can call it. -ffp-contract=off keeps
the compiler from fusing a*b+c into FMAs, so the arithmetic is exactly what the
source says. -fopenmp lets the per-gate scan run on several threads
(oracle_set_threads) with unchanged per-amplitude arithmetic.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
