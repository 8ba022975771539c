"""Continuous-batching server for circuit requests.

Requests (a register's dims and a gate list) arrive over time. The server keeps
admitted requests' statevectors resident on the GPU and advances all of them
together: every scheduler tick takes the next quantum of gates of every
resident request (more gates for smaller registers, so that each request's
share of a tick is about the same device work) and applies them in one batched
call (qd_batch_apply: one launch per round across all requests). A request that arrives while others
are running is admitted at the next tick as soon as a slot and enough of the
HBM budget are free; a finished request's memory is released at once. The host
prepares tick k+1 while the device runs tick k; completion is observed through
one HIP event per tick. A request's FP64 norm is enqueued right after its last
gates (qd_norm_noalloc, written by the device into pinned host memory), so
retiring it reads a finished value and never waits on the stream the other
requests share.

Per-request arithmetic does not depend on the mix: a fused pass applies each of
its gates with the same per-class arithmetic as a lone gate, so a request's
final state is bitwise the same whether it ran alone or among others, and
however its circuit was cut into quanta. With `reorder` > 0 each tick's passes
also take later gates of the quantum that commute with the gates they skip
(qd_circuit_options.reorder): fewer passes per tick, and a final state equal to
the in-order one up to rounding (the planned order depends on the quantum
boundaries, so bitwise equality with a solo run no longer holds).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional, Sequence

import numpy as np

from .binding import Batch, GateList, State, norm_noalloc


@dataclass
class ServeRequest:
    rid: int
    arrival: float                 # seconds after the server clock starts
    dims: Sequence[int]
    gates: GateList
    admitted: Optional[float] = None
    finished: Optional[float] = None
    norm: Optional[float] = None
    state: Optional[State] = None
    pos: int = 0                   # gates already enqueued
    done_tick: Optional[int] = None
    rejected: bool = False
    slot: int = -1                 # entry of the server's pinned norm buffer

    @property
    def D(self) -> int:
        return int(math.prod(self.dims))

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class Server:
    def __init__(self, precision: str = "c64", budget_bytes: float = 200e9, max_slots: int = 256,
                 quantum: int = 32, tile_amps: int = 0, min_run: int = 0, keep_states: bool = False,
                 tick_updates: float = 5e8, reorder: int = 0):
        import torch

        self.torch = torch
        self.precision = precision
        self.amp_bytes = 16 if precision == "c128" else 8
        self.budget = float(budget_bytes)
        self.max_slots = max_slots
        # Gates per request per tick: about tick_updates gate-amplitude updates
        # (a millisecond or so of device work), at least `quantum`. Small
        # requests then finish in one or a few ticks instead of len(gates) /
        # quantum ticks, each as long as the largest resident request's quantum.
        self.quantum = quantum
        self.tick_updates = tick_updates
        self.tile_amps, self.min_run, self.reorder = tile_amps, min_run, reorder
        self.keep_states = keep_states
        self.batch = Batch(precision)
        self.stream = torch.cuda.current_stream()
        self.resident: List[ServeRequest] = []
        self.queue: Deque[ServeRequest] = deque()
        self.finished: List[ServeRequest] = []
        self.resident_bytes = 0
        self.peak_bytes = 0
        self.ticks = 0
        self.events: Dict[int, object] = {}
        self.t0 = time.perf_counter()
        self.max_resident = 0
        # one pinned FP64 entry per slot: the device writes a finished request's
        # norm there, and the host reads it once the tick's event has completed
        self.norms = torch.zeros(max_slots, dtype=torch.float64, pin_memory=True)
        self.free_slots = list(range(max_slots - 1, -1, -1))

    def state_bytes(self, r: ServeRequest) -> int:
        return r.D * self.amp_bytes

    def submit(self, r: ServeRequest) -> None:
        if self.state_bytes(r) > self.budget:
            r.rejected = True  # can never fit: refuse instead of blocking the queue forever
            self.finished.append(r)
            return
        self.queue.append(r)

    def _admit(self, now: float) -> None:
        while self.queue and len(self.resident) < self.max_slots:
            r = self.queue[0]
            if self.resident_bytes + self.state_bytes(r) > self.budget:
                break  # FIFO: wait for memory to free up
            self.queue.popleft()
            r.state = State(r.dims, self.precision, init=0, stream=self.stream)
            r.slot = self.free_slots.pop()
            r.admitted = now
            self.resident.append(r)
            self.resident_bytes += self.state_bytes(r)
            self.peak_bytes = max(self.peak_bytes, self.resident_bytes)
            self.max_resident = max(self.max_resident, len(self.resident))

    def _retire(self, now: float) -> None:
        keep = []
        for r in self.resident:
            if r.done_tick is not None and self.events[r.done_tick].query():
                r.norm = float(self.norms[r.slot])  # FP64 norm on the host: the request is complete
                r.finished = time.perf_counter() - self.t0
                self.free_slots.append(r.slot)
                r.slot = -1
                if not self.keep_states:
                    r.state.close()
                    r.state = None
                self.resident_bytes -= self.state_bytes(r)
                self.finished.append(r)
            else:
                keep.append(r)
        self.resident = keep
        live = {r.done_tick for r in self.resident}
        for t in [t for t in self.events if t not in live and t < self.ticks - 4]:
            del self.events[t]

    def _tick(self) -> bool:
        """Enqueue the next quantum of every resident request, and the norm of every
        request whose gates are now all enqueued (an empty circuit included);
        False if there was nothing to enqueue."""
        work = [r for r in self.resident if r.pos < len(r.gates)]
        if work:
            lists = []
            for r in work:
                q = max(self.quantum, int(self.tick_updates // r.D))
                lists.append(r.gates.view(r.pos, q))  # no re-marshalling per tick
                r.pos += len(lists[-1])
            self.batch.apply([r.state for r in work], lists, tile_amps=self.tile_amps, min_run=self.min_run,
                             reorder=self.reorder)
        finishing = [r for r in self.resident if r.done_tick is None and r.pos >= len(r.gates)]
        if not work and not finishing:
            return False
        for r in finishing:
            norm_noalloc([r.state], self.norms[r.slot:r.slot + 1])
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.events[self.ticks] = ev
        for r in finishing:
            r.done_tick = self.ticks
        self.ticks += 1
        return True

    def run(self, requests: Sequence[ServeRequest], realtime: bool = True, timeout: float = 600.0,
            max_in_flight: int = 2) -> Dict:
        """Serve requests (sorted by arrival). With realtime, a request enters the
        queue when the wall clock reaches its arrival time; otherwise all are
        present at t = 0 (closed loop). At most max_in_flight ticks are queued on
        the device, so new arrivals join within a couple of ticks."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = self.t0 = time.perf_counter()
        while pending or self.queue or self.resident:
            now = time.perf_counter() - t0
            if now > timeout:
                raise TimeoutError("serving did not finish in time")
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.popleft()
                if not realtime:
                    r.arrival = 0.0
                self.submit(r)
            self._retire(now)
            self._admit(now)
            inflight = [t for t in self.events if t >= self.ticks - max_in_flight and not self.events[t].query()]
            if len(inflight) >= max_in_flight:
                self.events[min(inflight)].synchronize()
                continue
            if not self._tick():
                if self.resident:
                    self.stream.synchronize()  # all work enqueued; wait for completions
                elif pending and realtime:
                    time.sleep(min(1e-3, max(0.0, pending[0].arrival - (time.perf_counter() - t0))))
        return self.report(time.perf_counter() - t0)

    def report(self, wall: float) -> Dict:
        done = [r for r in self.finished if not r.rejected]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        buckets = {}
        for lo in range(3, 8):
            sel = [r.latency for r in done if 10 ** lo <= r.D < 10 ** (lo + 1) or (lo == 7 and r.D == 10 ** 8)]
            if sel:
                buckets[f"[1e{lo},1e{lo + 1})"] = {"n": len(sel), "p50_ms": 1e3 * float(np.percentile(sel, 50)),
                                                   "p99_ms": 1e3 * float(np.percentile(sel, 99))}
        return {"requests": len(done), "rejected": sum(r.rejected for r in self.finished), "wall_s": wall,
                "throughput_rps": len(done) / wall if wall > 0 else None,
                "p50_ms": 1e3 * float(np.percentile(lat, 50)) if lat.size else None,
                "p99_ms": 1e3 * float(np.percentile(lat, 99)) if lat.size else None,
                "buckets": buckets, "ticks": self.ticks, "peak_resident_GB": self.peak_bytes / 1e9,
                "max_resident_requests": self.max_resident,
                "budget_GB": self.budget / 1e9}

    def close(self) -> None:
        for r in self.resident:
            if r.state is not None:
                r.state.close()
        self.batch.close()


def requests_from_specs(reqs) -> List[ServeRequest]:
    """ServeRequests from qd_inputs.circuits.Request records."""
    return [ServeRequest(r.rid, r.arrival, list(r.spec.dims), GateList(r.spec.gates())) for r in reqs]
