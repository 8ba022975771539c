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


# Built with AddressSanitizer and UndefinedBehaviorSanitizer (and no OpenMP, whose
# runtime the sanitizers do not follow) when the oracle itself is under test:
# load it with QD_ORACLE_LIB=<path> and gcc's libasan/libubsan preloaded.
LIB_SANITIZED = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SANITIZED if sanitize else LIB
    flags = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas"] if sanitize else ["-O2", "-fopenmp"])
    cmd = ["gcc", *flags, "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
