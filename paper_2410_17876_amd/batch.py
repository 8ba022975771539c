"""Batched execution of many independent circuits (qd_batch_apply).

A BatchRunner owns one state per circuit and advances all of them together:
each circuit is split into fused passes, and round r is one launch that runs
pass r of every circuit still running. Circuits whose register fits one tile
run entirely in one round, in LDS. Results are bitwise those of running each
circuit alone with the same tile options.
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

from .binding import Batch, BatchPlan, GateList, State


class BatchRunner:
    def __init__(self, dims_list: Sequence[Sequence[int]], precision="c64", device=None, stream=None):
        self.precision = precision
        self.states: List[State] = [State(d, precision, device=device, stream=stream) for d in dims_list]
        self.batch = Batch(precision)

    def reset(self) -> None:
        for st in self.states:
            st.reset(0)

    def run(self, gate_lists: Sequence, tile_amps: int = 0, min_run: int = 0, reorder: int = 0) -> dict:
        """Apply gate_lists[i] to state i; returns rounds/items and wall time (synchronised)."""
        gls = [g if isinstance(g, GateList) else GateList(g) for g in gate_lists]
        t0 = time.perf_counter()
        info = self.batch.apply(self.states, gls, tile_amps=tile_amps, min_run=min_run, reorder=reorder)
        self.states[0].synchronize()
        info["seconds"] = time.perf_counter() - t0
        return info

    def compile(self, gate_lists: Sequence, tile_amps: int = 0, min_run: int = 0, reorder: int = 0) -> BatchPlan:
        """Plan and upload the rounds once; replay them with plan.run(graph=...)."""
        return BatchPlan(self.states, gate_lists, tile_amps=tile_amps, min_run=min_run, reorder=reorder)

    def updates(self, gate_lists) -> int:
        """Gate-amplitude updates of the gate lists (as counted per gate by the library)."""
        from .binding import gate_info
        total = 0
        for st, gl in zip(self.states, gate_lists):
            for g in (gl.gates if isinstance(gl, GateList) else gl):
                total += gate_info(st.dims, g.targets, g.U, g.controls, g.values, self.precision)["updated"]
        return total

    def close(self) -> None:
        for st in self.states:
            st.close()
        self.batch.close()
