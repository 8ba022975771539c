"""ctypes binding of libqd (include/qd.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels. torch supplies
device memory (the amplitude buffer is a torch tensor wrapped through
qd_state_create_external) and the stream (torch's current stream), nothing else.
There is no fallback: if libqd.so is missing or cannot be loaded, importing
this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QD_LIBQD selects another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("QD_LIBQD", os.path.join(HERE, "libqd.so"))

QD_C64, QD_C128 = 1, 2
QD_DEVICE, QD_HOST = 0, 1
STATUS = {0: "QD_OK", -1: "QD_ERR_INVALID_ARGUMENT", -2: "QD_ERR_DIM_OVERFLOW", -3: "QD_ERR_OUT_OF_MEMORY",
          -4: "QD_ERR_DEVICE", -5: "QD_ERR_NOT_SUPPORTED", -6: "QD_ERR_BUFFER_TOO_SMALL"}
PRECISIONS = {"c64": QD_C64, "c128": QD_C128, QD_C64: QD_C64, QD_C128: QD_C128}


class QDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GateDesc(C.Structure):
    _fields_ = [("targets", C.POINTER(C.c_int32)), ("k", C.c_int32), ("controls", C.POINTER(C.c_int32)),
                ("values", C.POINTER(C.c_int32)), ("m", C.c_int32), ("U", C.POINTER(C.c_double))]


class CircuitOptions(C.Structure):
    _fields_ = [("fuse", C.c_int32), ("tile_amps", C.c_int32), ("min_run", C.c_int32), ("reorder", C.c_int32),
                ("passes", C.c_int32), ("fused_passes", C.c_int32)]


class GateInfo(C.Structure):
    _fields_ = [("kernel", C.c_char * 64), ("category", C.c_int32), ("M", C.c_int32), ("classes", C.c_uint64),
                ("updated", C.c_uint64), ("bytes", C.c_uint64), ("flops", C.c_uint64)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2410_17876_amd/build.py (or __graft_entry__.build())")
    # torch first: its bundled HIP runtime then satisfies libqd's libamdhip64
    # dependency, so both share one runtime (and one device context). Loaded the
    # other way round, the process holds two HIP runtimes, and the second one to
    # initialise does not see the GPU.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    i32p = C.POINTER(C.c_int32)
    f64p = C.POINTER(C.c_double)
    u64p = C.POINTER(C.c_uint64)
    vp = C.c_void_p
    sig = {
        "qd_dim": [i32p, C.c_int32, u64p],
        "qd_check_gate": [i32p, C.c_int32, i32p, C.c_int32, i32p, i32p, C.c_int32],
        "qd_gate_info_for": [i32p, C.c_int32, C.c_int32, i32p, C.c_int32, i32p, i32p, C.c_int32, f64p,
                             C.POINTER(GateInfo)],
        "qd_class_bases": [i32p, C.c_int32, i32p, C.c_int32, i32p, i32p, C.c_int32, C.c_uint64, C.c_uint64, u64p],
        "qd_state_create": [i32p, C.c_int32, C.c_int32, C.POINTER(vp)],
        "qd_state_create_external": [i32p, C.c_int32, C.c_int32, vp, C.c_uint64, C.POINTER(vp)],
        "qd_state_destroy": [vp],
        "qd_state_set_stream": [vp, vp],
        "qd_state_reset": [vp, C.c_uint64],
        "qd_state_set_amplitudes": [vp, f64p, C.c_uint64, C.c_uint64],
        "qd_state_get_amplitudes": [vp, f64p, C.c_uint64, C.c_uint64],
        "qd_state_info": [vp, u64p, i32p, C.POINTER(vp)],
        "qd_apply_gate": [vp, i32p, C.c_int32, i32p, i32p, C.c_int32, f64p],
        "qd_apply_gate_masked": [vp, i32p, C.c_int32, i32p, C.POINTER(C.c_uint32), C.c_int32, f64p],
        "qd_sparse_dim": [i32p, C.c_int32, u64p, u64p, i32p],
        "qd_sparse_create": [i32p, C.c_int32, C.POINTER(vp)],
        "qd_sparse_destroy": [vp],
        "qd_sparse_set_stream": [vp, vp],
        "qd_sparse_apply_gate": [vp, i32p, C.c_int32, i32p, i32p, C.c_int32, f64p],
        "qd_sparse_apply_circuit": [vp, C.POINTER(GateDesc), C.c_int32],
        "qd_sparse_nnz": [vp, u64p],
        "qd_sparse_get": [vp, u64p, f64p, C.c_uint64],
        "qd_sparse_get_wide": [vp, u64p, f64p, C.c_uint64],
        "qd_norm": [vp, f64p],
        "qd_norm_noalloc": [C.POINTER(vp), C.c_int32, vp],
        "qd_probabilities": [vp, f64p, C.c_uint64, C.c_int32],
        "qd_synchronize": [vp],
        "qd_copy_ceiling": [vp, C.c_int32, f64p],
        "qd_apply_circuit": [vp, C.POINTER(GateDesc), C.c_int32, C.POINTER(CircuitOptions)],
        "qd_circuit_plan": [i32p, C.c_int32, C.c_int32, C.POINTER(GateDesc), C.c_int32, C.POINTER(CircuitOptions),
                            i32p, i32p, i32p, i32p],
        "qd_batch_create": [C.c_int32, C.POINTER(vp)],
        "qd_batch_destroy": [vp],
        "qd_batch_apply": [vp, C.POINTER(vp), C.POINTER(C.POINTER(GateDesc)), i32p, C.c_int32,
                           C.POINTER(CircuitOptions)],
        "qd_batch_compile": [C.POINTER(vp), C.POINTER(C.POINTER(GateDesc)), i32p, C.c_int32,
                             C.POINTER(CircuitOptions), C.POINTER(vp)],
        "qd_batch_plan_run": [vp, C.c_int32],
        "qd_batch_plan_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.qd_last_error.argtypes = []
    L.qd_last_error.restype = C.c_char_p
    L.qd_version.argtypes = []
    L.qd_version.restype = C.c_char_p
    return L


lib = _load()


def check(rc: int) -> int:
    if rc != 0:
        raise QDError(rc, lib.qd_last_error().decode(errors="replace"))
    return rc


def _i32(x: Sequence[int]):
    a = np.ascontiguousarray(np.asarray(list(x) or [0], dtype=np.int32))
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _u(U) -> tuple:
    a = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("U must be a square matrix")
    return a, a.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))


class GateList:
    """A gate list marshalled once into qd_gate_desc records (keeps the arrays alive)."""

    def __init__(self, gates):
        self.gates = list(gates)
        self._keep = []
        self.descs = (GateDesc * max(1, len(self.gates)))()
        for i, g in enumerate(self.gates):
            t, tp = _i32(g.targets)
            c, cp = _i32(g.controls)
            v, vp_ = _i32(g.values)
            u, up = _u(g.U)
            self._keep += [t, c, v, u]
            self.descs[i] = GateDesc(tp, len(g.targets), cp, vp_, len(g.controls), up)

    def __len__(self):
        return len(self.gates)

    def view(self, start: int, count: int) -> "GateListView":
        """Gates [start, start + count) without marshalling them again."""
        start = max(0, min(start, len(self.gates)))
        count = max(0, min(count, len(self.gates) - start))
        return GateListView(self, start, count)


class GateListView:
    """A contiguous range of a GateList's records (shares its arrays)."""

    def __init__(self, parent: GateList, start: int, count: int):
        self.parent = parent
        self.count = count
        self.gates = parent.gates[start:start + count]
        self.descs = C.cast(C.addressof(parent.descs) + start * C.sizeof(GateDesc), C.POINTER(GateDesc))

    def __len__(self):
        return self.count


def _options(fuse=True, tile_amps=0, min_run=0, reorder=0) -> CircuitOptions:
    return CircuitOptions(1 if fuse else 0, int(tile_amps), int(min_run), int(reorder), 0, 0)


def circuit_plan(dims, gates, precision="c128", fuse=True, tile_amps=0, min_run=0, reorder=0, with_order=False):
    """Passes qd_apply_circuit would enqueue: list of (gates in pass, tile amplitudes or 0);
    with_order: also the applied gates' indices in application order."""
    gl = gates if isinstance(gates, GateList) else GateList(gates)
    d, dp = _i32(dims)
    n = len(gl)
    pg = np.zeros(max(1, n), dtype=np.int32)
    pt = np.zeros(max(1, n), dtype=np.int32)
    order = np.zeros(max(1, n), dtype=np.int32)
    npass = C.c_int32()
    opts = _options(fuse, tile_amps, min_run, reorder)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    check(lib.qd_circuit_plan(dp, len(dims), PRECISIONS[precision], gl.descs, n, C.byref(opts),
                              ptr(pg), ptr(pt), ptr(order), C.byref(npass)))
    passes = [(int(pg[i]), int(pt[i])) for i in range(npass.value)]
    if with_order:
        return passes, [int(x) for x in order[:sum(p[0] for p in passes)]]
    return passes


def dim(dims: Sequence[int]) -> int:
    d, dp = _i32(dims)
    out = C.c_uint64()
    check(lib.qd_dim(dp, len(dims), C.byref(out)))
    return out.value


def check_gate(dims, targets, controls=(), values=()) -> None:
    d, dp = _i32(dims)
    t, tp = _i32(targets)
    c, cp = _i32(controls)
    v, vp_ = _i32(values)
    check(lib.qd_check_gate(dp, len(dims), tp, len(targets), cp, vp_, len(controls)))


def gate_info(dims, targets, U, controls=(), values=(), precision="c128") -> dict:
    d, dp = _i32(dims)
    t, tp = _i32(targets)
    c, cp = _i32(controls)
    v, vp_ = _i32(values)
    u, up = _u(U)
    info = GateInfo()
    check(lib.qd_gate_info_for(dp, len(dims), PRECISIONS[precision], tp, len(targets), cp, vp_, len(controls), up,
                               C.byref(info)))
    return {"kernel": info.kernel.decode(), "category": info.category, "M": info.M, "classes": info.classes,
            "updated": info.updated, "bytes": info.bytes, "flops": info.flops}


def class_bases(dims, targets, controls=(), values=(), first=0, count=None) -> np.ndarray:
    d, dp = _i32(dims)
    t, tp = _i32(targets)
    c, cp = _i32(controls)
    v, vp_ = _i32(values)
    if count is None:
        M = int(np.prod([dims[x] for x in targets]))
        cpd = int(np.prod([dims[x] for x in controls])) if controls else 1
        count = dim(dims) // (M * cpd) - first
    out = np.empty(max(1, count), dtype=np.uint64)
    check(lib.qd_class_bases(dp, len(dims), tp, len(targets), cp, vp_, len(controls), first, count,
                             out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out[:count]


class State:
    """A statevector resident on the GPU.

    The amplitude buffer is a torch tensor (``self.buffer``: float64 pairs for
    c128, float32 pairs for c64); work runs on the torch stream current at
    creation (or the one given).
    """

    def __init__(self, dims: Sequence[int], precision="c128", device=None, init: Optional[int] = 0, stream=None):
        import torch

        self.dims = [int(x) for x in dims]
        self.precision = PRECISIONS[precision]
        self.D = dim(self.dims)
        self.device = torch.device(device if device is not None else "cuda")
        dt = torch.float64 if self.precision == QD_C128 else torch.float32
        self.buffer = torch.empty(2 * self.D, dtype=dt, device=self.device)
        self._h = C.c_void_p()
        d, dp = _i32(self.dims)
        with torch.cuda.device(self.device):
            check(lib.qd_state_create_external(dp, len(self.dims), self.precision, C.c_void_p(self.buffer.data_ptr()),
                                               self.buffer.numel() * self.buffer.element_size(), C.byref(self._h)))
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            check(lib.qd_state_set_stream(self._h, C.c_void_p(self.stream.cuda_stream)))
            if init is not None:
                self.reset(init)

    @property
    def handle(self):
        return self._h

    def reset(self, j: int = 0) -> "State":
        check(lib.qd_state_reset(self._h, int(j)))
        return self

    def apply(self, targets, U, controls=(), values=()) -> "State":
        t, tp = _i32(targets)
        c, cp = _i32(controls)
        v, vp_ = _i32(values)
        u, up = _u(U)
        check(lib.qd_apply_gate(self._h, tp, len(targets), cp, vp_, len(controls), up))
        return self

    def apply_masked(self, targets, U, controls=(), masks=()) -> "State":
        """Apply U on the classes whose digit at controls[l] is in the set bit mask masks[l] (qd_apply_gate_masked)."""
        t, tp = _i32(targets)
        c, cp = _i32(controls)
        mk = np.ascontiguousarray(np.asarray(list(masks) or [0], dtype=np.uint32))
        u, up = _u(U)
        check(lib.qd_apply_gate_masked(self._h, tp, len(targets), cp, mk.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       len(controls), up))
        return self

    def apply_gate(self, g) -> "State":
        return self.apply(g.targets, g.U, g.controls, g.values)

    def run(self, gates) -> "State":
        for g in gates:
            self.apply_gate(g)
        return self

    def run_circuit(self, gates, fuse=True, tile_amps=0, min_run=0, reorder=0) -> dict:
        """Apply a gate list through qd_apply_circuit; returns the pass counts."""
        gl = gates if isinstance(gates, GateList) else GateList(gates)
        opts = _options(fuse, tile_amps, min_run, reorder)
        check(lib.qd_apply_circuit(self._h, gl.descs, len(gl), C.byref(opts)))
        return {"passes": opts.passes, "fused_passes": opts.fused_passes}

    def norm(self) -> float:
        out = C.c_double()
        check(lib.qd_norm(self._h, C.byref(out)))
        return out.value

    def probabilities(self, location: str = "device"):
        """p_j = |a_j|^2 in FP64: a torch tensor on the device, or a numpy array."""
        import torch

        if location == "device":
            out = torch.empty(self.D, dtype=torch.float64, device=self.device)
            check(lib.qd_probabilities(self._h, C.cast(C.c_void_p(out.data_ptr()), C.POINTER(C.c_double)), self.D,
                                       QD_DEVICE))
            return out
        out = np.empty(self.D, dtype=np.float64)
        check(lib.qd_probabilities(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), self.D, QD_HOST))
        return out

    def amplitudes(self, offset: int = 0, count: Optional[int] = None) -> np.ndarray:
        """Amplitudes [offset, offset+count) as complex128 on the host."""
        count = self.D - offset if count is None else count
        out = np.empty(count, dtype=np.complex128)
        check(lib.qd_state_get_amplitudes(self._h, out.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                          offset, count))
        return out

    def set_amplitudes(self, values, offset: int = 0) -> "State":
        v = np.ascontiguousarray(np.asarray(values, dtype=np.complex128))
        check(lib.qd_state_set_amplitudes(self._h, v.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                          offset, v.size))
        return self

    def set_interleaved(self, values: np.ndarray, offset: int = 0) -> "State":
        """Upload FP64 interleaved (re, im) values starting at amplitude ``offset``."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        check(lib.qd_state_set_amplitudes(self._h, v.ctypes.data_as(C.POINTER(C.c_double)), offset, v.size // 2))
        return self

    def copy_ceiling(self, reps: int = 3) -> float:
        """Fastest in-place read+rewrite pass over the state, in ms (values unchanged)."""
        out = C.c_double()
        check(lib.qd_copy_ceiling(self._h, int(reps), C.byref(out)))
        return out.value

    def synchronize(self) -> None:
        check(lib.qd_synchronize(self._h))

    def close(self) -> None:
        if self._h:
            lib.qd_state_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def norm_noalloc(states, out) -> None:
    """qd_norm_noalloc: enqueue the FP64 norms of `states` into `out`, a float64
    torch tensor on their device (or a pinned host tensor) with room for one
    value per state; allocates nothing and does not wait (read `out` after the
    states' streams have reached this call)."""
    hs = (C.c_void_p * max(1, len(states)))(*[st.handle for st in states])
    check(lib.qd_norm_noalloc(hs, len(states), C.c_void_p(out.data_ptr())))


def _batch_args(states, gate_lists):
    n = len(states)
    if len(gate_lists) != n:
        raise ValueError("one gate list per state")
    gls = [g if isinstance(g, (GateList, GateListView)) else GateList(g) for g in gate_lists]
    hs = (C.c_void_p * max(1, n))(*[st.handle for st in states])
    gp = (C.POINTER(GateDesc) * max(1, n))(*[C.cast(g.descs, C.POINTER(GateDesc)) for g in gls])
    counts = np.array([len(g) for g in gls] or [0], dtype=np.int32)
    return gls, hs, gp, counts


def sparse_dim(dims) -> tuple:
    """(D, key words) of a sparse register: D = prod dims as a Python int (< 2^127)."""
    d, dp = _i32(dims)
    lo, hi, w = C.c_uint64(), C.c_uint64(), C.c_int32()
    check(lib.qd_sparse_dim(dp, len(dims), C.byref(lo), C.byref(hi), C.byref(w)))
    return (hi.value << 64) | lo.value, w.value


class SparseState:
    """A sparse statevector (qd_sparse_*): nonzero amplitudes as (basis index, complex128) pairs on the GPU.

    Gates run on the torch stream current at creation (or the one given)."""

    def __init__(self, dims, stream=None):
        import torch

        self.dims = [int(d) for d in dims]
        self.D, self.words = sparse_dim(self.dims)
        d, dp = _i32(self.dims)
        self._h = C.c_void_p()
        check(lib.qd_sparse_create(dp, len(self.dims), C.byref(self._h)))
        st = stream if stream is not None else torch.cuda.current_stream()
        check(lib.qd_sparse_set_stream(self._h, C.c_void_p(st.cuda_stream)))

    def apply(self, targets, U, controls=(), values=()) -> "SparseState":
        t, tp = _i32(targets)
        c, cp = _i32(controls)
        v, vp_ = _i32(values)
        u, up = _u(U)
        check(lib.qd_sparse_apply_gate(self._h, tp, len(targets), cp, vp_, len(controls), up))
        return self

    def apply_gate(self, g) -> "SparseState":
        return self.apply(g.targets, g.U, g.controls, g.values)

    def run(self, gates) -> "SparseState":
        """Apply a gate list in one call (qd_sparse_apply_circuit)."""
        gl = gates if isinstance(gates, GateList) else GateList(gates)
        check(lib.qd_sparse_apply_circuit(self._h, gl.descs, len(gl)))
        return self

    def nnz(self) -> int:
        out = C.c_uint64()
        check(lib.qd_sparse_nnz(self._h, C.byref(out)))
        return out.value

    def entries(self):
        """(keys, amplitudes complex128) in increasing basis index: keys is a uint64
        array when D < 2^64, else a list of Python ints."""
        n = self.nnz()
        amps = np.zeros(2 * max(1, n), dtype=np.float64)
        if self.D < 2**64:
            keys = np.zeros(max(1, n), dtype=np.uint64)
            check(lib.qd_sparse_get(self._h, keys.ctypes.data_as(C.POINTER(C.c_uint64)),
                                    amps.ctypes.data_as(C.POINTER(C.c_double)), n))
            return keys[:n], amps.view(np.complex128)[:n]
        halves = np.zeros(2 * max(1, n), dtype=np.uint64)
        check(lib.qd_sparse_get_wide(self._h, halves.ctypes.data_as(C.POINTER(C.c_uint64)),
                                     amps.ctypes.data_as(C.POINTER(C.c_double)), n))
        keys = [(int(halves[2 * i + 1]) << 64) | int(halves[2 * i]) for i in range(n)]
        return keys, amps.view(np.complex128)[:n]

    def close(self) -> None:
        if self._h:
            lib.qd_sparse_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """A compiled batch (qd_batch_compile): replay the same gate lists on the states."""

    def __init__(self, states, gate_lists, tile_amps=0, min_run=0, reorder=0):
        self.states = list(states)
        self._keep = _batch_args(self.states, gate_lists)
        gls, hs, gp, counts = self._keep
        opts = _options(True, tile_amps, min_run, reorder)
        self._h = C.c_void_p()
        check(lib.qd_batch_compile(hs, gp, counts.ctypes.data_as(C.POINTER(C.c_int32)), len(self.states),
                                   C.byref(opts), C.byref(self._h)))
        self.rounds, self.items = opts.passes, opts.fused_passes

    def run(self, graph: bool = False) -> None:
        check(lib.qd_batch_plan_run(self._h, 1 if graph else 0))

    def close(self) -> None:
        if self._h:
            lib.qd_batch_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch context (qd_batch): advances many independent states together."""

    def __init__(self, precision="c128"):
        self.precision = PRECISIONS[precision]
        self._h = C.c_void_p()
        check(lib.qd_batch_create(self.precision, C.byref(self._h)))

    def apply(self, states, gate_lists, tile_amps=0, min_run=0, reorder=0) -> dict:
        """Apply gate_lists[i] to states[i] for all i (qd_batch_apply)."""
        n = len(states)
        gls, hs, gp, counts = _batch_args(states, gate_lists)
        opts = _options(True, tile_amps, min_run, reorder)
        check(lib.qd_batch_apply(self._h, hs, gp, counts.ctypes.data_as(C.POINTER(C.c_int32)), n, C.byref(opts)))
        return {"rounds": opts.passes, "items": opts.fused_passes}

    def close(self) -> None:
        if self._h:
            lib.qd_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

