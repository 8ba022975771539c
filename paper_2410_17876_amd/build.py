"""Build libqd.so (the HIP library behind include/qd.h) for gfx950, in-tree.

Each source under csrc/ is compiled by hipcc into _build/, then linked into
paper_2410_17876_amd/libqd.so. Packed FP32 instructions are disabled for all
device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqd.so")
ARCH = os.environ.get("QD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["abi.cpp", "planner.cpp", "fusion.cpp", "sweep.hip", "fused.hip", "mfma.hip", "reduce.hip", "sparse.hip"]

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, verbose: bool, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + (".san.o" if extra else ".o"))
    cmd = [_hipcc(), *CFLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


# The host code built with AddressSanitizer and UndefinedBehaviorSanitizer (the
# device code is built as always): load it with QD_LIBQD=<path> and clang's
# ASan runtime preloaded, to check the ABI's host logic.
LIB_SANITIZED = os.path.join(HERE, "libqd_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    extra = SAN_FLAGS if sanitize else []
    with ThreadPoolExecutor(min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, extra), SOURCES))
    lib = LIB_SANITIZED if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *extra, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
