"""CPU FP64 oracle for mixed-radix qudit statevector simulation.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are its only users. It never imports the GPU
package, and the GPU package never imports it.

The arithmetic lives in qd_oracle.c (see its header for the paper passages each
step follows); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QD_ORACLE_LIB", _build.LIB)  # e.g. the sanitizer build
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.oracle_dim.argtypes = [C.c_int, i32p]
        L.oracle_dim.restype = C.c_int64
        L.oracle_init_zero.argtypes = [C.c_int, i32p, f64p]
        L.oracle_apply.argtypes = [C.c_int, i32p, f64p, C.c_int, i32p, C.c_int, i32p, i32p, f64p]
        L.oracle_apply_masked.argtypes = [C.c_int, i32p, f64p, C.c_int, i32p, C.c_int, i32p,
                                          np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS"), f64p]
        L.oracle_class_members.argtypes = [C.c_int, i32p, C.c_int, i32p, C.c_int, i32p, i32p,
                                           C.c_int64, i64p, i64p, i32p]
        L.oracle_rows.argtypes = [C.c_int, f64p, C.c_int64, f64p, i32p, f64p]
        L.oracle_norm.argtypes = [C.c_int64, f64p, C.POINTER(C.c_double)]
        L.oracle_probabilities.argtypes = [C.c_int64, f64p, f64p]
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_get_threads.argtypes = []
        for f in (L.oracle_init_zero, L.oracle_apply, L.oracle_apply_masked, L.oracle_class_members, L.oracle_rows,
                  L.oracle_norm, L.oracle_probabilities, L.oracle_set_threads, L.oracle_get_threads):
            f.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads for the per-gate scans (the result is bitwise the same for any count)."""
    if lib().oracle_set_threads(int(n)) != 0:
        raise ValueError("thread count must be >= 1")


def get_threads() -> int:
    return int(lib().oracle_get_threads())


class threads:
    """Context manager: run the enclosed oracle calls on n threads."""

    def __init__(self, n: int):
        self.n = int(n)

    def __enter__(self):
        self.prev = get_threads()
        set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def _i32(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(list(x), dtype=np.int32))
    return a if a.size else np.zeros(1, dtype=np.int32)


def _u(U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    return U.view(np.float64).reshape(-1)


def dim(dims: Sequence[int]) -> int:
    return int(lib().oracle_dim(len(dims), _i32(dims)))


def zero_state(dims: Sequence[int]) -> np.ndarray:
    D = dim(dims)
    if D < 0:
        raise ValueError("invalid dims")
    psi = np.empty(2 * D, dtype=np.float64)
    if lib().oracle_init_zero(len(dims), _i32(dims), psi) != 0:
        raise ValueError("invalid dims")
    return psi.view(np.complex128)


def apply(dims, psi: np.ndarray, targets, U, controls=(), values=()) -> np.ndarray:
    """Apply one gate to the complex128 statevector ``psi`` in place; returns psi."""
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous:
        raise TypeError("psi must be a contiguous complex128 array")
    rc = lib().oracle_apply(len(dims), _i32(dims), psi.view(np.float64), len(targets), _i32(targets),
                            len(controls), _i32(controls), _i32(values), _u(U))
    if rc != 0:
        raise ValueError("invalid gate")
    return psi


def apply_masked(dims, psi: np.ndarray, targets, U, controls=(), masks=()) -> np.ndarray:
    """Apply a gate whose control l accepts the values in bit mask masks[l], in place; returns psi."""
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous:
        raise TypeError("psi must be a contiguous complex128 array")
    mk = np.ascontiguousarray(np.asarray(masks, dtype=np.uint32).reshape(-1)) if len(masks) else np.zeros(1, np.uint32)
    rc = lib().oracle_apply_masked(len(dims), _i32(dims), psi.view(np.float64), len(targets), _i32(targets),
                                   len(controls), _i32(controls), mk, _u(U))
    if rc != 0:
        raise ValueError("invalid gate")
    return psi


def apply_gate(dims, psi, g) -> np.ndarray:
    return apply(dims, psi, g.targets, g.U, g.controls, g.values)


def run(dims, gates, psi=None) -> np.ndarray:
    """Run a gate list from |0..0> (or from a copy of ``psi``)."""
    psi = zero_state(dims) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    for g in gates:
        apply_gate(dims, psi, g)
    return psi


def class_members(dims, targets, controls, values, out_idx):
    """Input addresses each sampled output amplitude depends on, and its row."""
    out_idx = np.ascontiguousarray(np.asarray(out_idx, dtype=np.int64))
    M = int(np.prod([dims[t] for t in targets]))
    members = np.empty(out_idx.size * M, dtype=np.int64)
    row = np.empty(max(1, out_idx.size), dtype=np.int32)
    rc = lib().oracle_class_members(len(dims), _i32(dims), len(targets), _i32(targets), len(controls),
                                    _i32(controls), _i32(values), out_idx.size, out_idx, members, row)
    if rc != 0:
        raise ValueError("invalid gate or index")
    return members.reshape(out_idx.size, M), row[: out_idx.size]


def rows(U, x: np.ndarray, row: np.ndarray) -> np.ndarray:
    """New amplitudes from gathered class inputs x (nsamp x M complex128)."""
    U = np.asarray(U, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty(x.shape[0], dtype=np.complex128)
    rc = lib().oracle_rows(U.shape[0], _u(U), x.shape[0], x.view(np.float64).reshape(-1),
                           np.ascontiguousarray(row, dtype=np.int32), out.view(np.float64))
    if rc != 0:
        raise ValueError("invalid rows")
    return out


def apply_sampled(dims, gate, out_idx, input_values) -> np.ndarray:
    """New amplitudes at ``out_idx`` after ``gate``, where ``input_values(idx)``
    returns the pre-gate amplitudes at any indices."""
    members, row = class_members(dims, gate.targets, gate.controls, gate.values, out_idx)
    x = input_values(members.reshape(-1)).reshape(members.shape)
    return rows(gate.U, x, row)


def norm(psi: np.ndarray) -> float:
    out = C.c_double()
    if lib().oracle_norm(psi.size, np.ascontiguousarray(psi).view(np.float64), C.byref(out)) != 0:
        raise ValueError("empty state")
    return out.value


def probabilities(psi: np.ndarray) -> np.ndarray:
    out = np.empty(psi.size, dtype=np.float64)
    if lib().oracle_probabilities(psi.size, np.ascontiguousarray(psi).view(np.float64), out) != 0:
        raise ValueError("empty state")
    return out
