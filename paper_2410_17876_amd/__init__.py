"""MI355X (gfx950) block simulation of mixed-radix qudit statevectors.

Implements the block-simulation method of arXiv 2410.17876 ("Fast classical
simulation of qubit-qudit hybrid systems") as HIP kernels behind the C ABI in
include/qd.h. This package is the Python binding of that library.
"""
from .binding import (QD_C128, QD_C64, Batch, BatchPlan, GateInfo, GateList, QDError, SparseState, State, check_gate,
                      circuit_plan, class_bases, dim, gate_info, lib, LIB_PATH, sparse_dim)

__all__ = ["Batch", "BatchPlan", "State", "SparseState", "QDError", "GateInfo", "GateList", "circuit_plan", "dim",
           "sparse_dim", "check_gate", "gate_info", "class_bases", "lib", "LIB_PATH", "QD_C64", "QD_C128"]
from . import batch, serve, tune  # noqa: E402  (batched runner, server, tile autotuner)
