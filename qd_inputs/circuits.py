"""Seeded gate-list generators for the workload configurations.

Every generator takes a seed and returns plain ``Gate`` records (see gates.py);
they never touch a statevector. The paper's own workloads are QASMBench circuits
(Sec. 3) that are not available here, so these synthetic circuits stand in for
them, with the gate categories of Sec. 2 (phase, permutation, superposition,
controlled):

  plain     dims [2,2,2,2,3,3] (D = 144), 200 gates of the *basic mix*
  large     dims 2^14 x 3^8 x 4^2 (D = 1.72e9), 500 gates: w.p. 0.1 a 2-qudit
            Haar unitary on a random ordered pair of distinct qudits, else the
            basic mix
  batched   512 circuits of 6..16 qudits, d uniform in {2,3,4,5}, D <= 1e6,
            depth uniform in 100..1000, basic mix
  served    request sizes log-uniform in [1e3, 1e8] amplitudes, d in 2..7,
            depth 50..500, basic mix, Poisson arrivals
  fused     12 ququints (D = 5^12), 300 Haar gates on 2 or 3 distinct qudits

The *basic mix* (one gate): w.p. 0.6 a 1-qudit Haar unitary on a uniform
target; w.p. 0.2 one of {generalized DFT, X_{+1}, Z} (1/3 each) on a uniform
target; w.p. 0.2 a controlled X_{+1}: an ordered pair (control, target) of
distinct qudits, control value uniform in 0..d_c-1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from .gates import Gate, clock, dft, haar, shift

SEEDS = {"plain": 1000, "large": 1001, "batched": 1002, "served": 1003, "fused": 1004}

PLAIN_DIMS = [2, 2, 2, 2, 3, 3]
LARGE_DIMS = [2] * 14 + [3] * 8 + [4] * 2
FUSED_DIMS = [5] * 12


def mix_gate(rng: np.random.Generator, dims: Sequence[int]) -> Gate:
    """One gate of the basic mix on a register with the given dims."""
    n = len(dims)
    r = rng.random()
    if r < 0.6 or (r >= 0.8 and n < 2):
        t = int(rng.integers(n))
        return Gate((t,), haar(dims[t], rng), kind="haar1")
    if r < 0.8:
        t = int(rng.integers(n))
        which = int(rng.integers(3))
        d = dims[t]
        if which == 0:
            return Gate((t,), dft(d), kind="dft")
        if which == 1:
            return Gate((t,), shift(d, 1), kind="x")
        return Gate((t,), clock(d), kind="z")
    c, t = (int(x) for x in rng.choice(n, 2, replace=False))
    v = int(rng.integers(dims[c]))
    return Gate((t,), shift(dims[t], 1), (c,), (v,), kind="cx")


def random_circuit(dims: Sequence[int], n_gates: int, seed: int) -> List[Gate]:
    rng = np.random.default_rng(seed)
    return [mix_gate(rng, dims) for _ in range(n_gates)]


def plain(seed: int = SEEDS["plain"], n_gates: int = 200):
    return list(PLAIN_DIMS), random_circuit(PLAIN_DIMS, n_gates, seed)


def large_gates(dims: Sequence[int], n_gates: int, seed: int) -> List[Gate]:
    rng = np.random.default_rng(seed)
    n = len(dims)
    out = []
    for _ in range(n_gates):
        if rng.random() < 0.1:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(Gate((a, b), haar(dims[a] * dims[b], rng), kind="haar2"))
        else:
            out.append(mix_gate(rng, dims))
    return out


def large(seed: int = SEEDS["large"], n_gates: int = 500, dims: Sequence[int] = LARGE_DIMS):
    return list(dims), large_gates(dims, n_gates, seed)


def fused_gates(dims: Sequence[int], n_gates: int, seed: int) -> List[Gate]:
    rng = np.random.default_rng(seed)
    n = len(dims)
    out = []
    for _ in range(n_gates):
        k = 2 if rng.random() < 0.5 else 3
        ts = [int(x) for x in rng.choice(n, k, replace=False)]
        M = int(np.prod([dims[t] for t in ts]))
        out.append(Gate(tuple(ts), haar(M, rng), kind=f"haar{k}"))
    return out


def fused(seed: int = SEEDS["fused"], n_gates: int = 300, dims: Sequence[int] = FUSED_DIMS):
    return list(dims), fused_gates(dims, n_gates, seed)


@dataclass
class CircuitSpec:
    dims: List[int]
    depth: int
    seed: int

    @property
    def D(self) -> int:
        return int(np.prod(self.dims))

    def gates(self) -> List[Gate]:
        return random_circuit(self.dims, self.depth, self.seed)


def batched_specs(seed: int = SEEDS["batched"], count: int = 512, cap: int = 10**6,
                  depth_lo: int = 100, depth_hi: int = 1000) -> List[CircuitSpec]:
    """Dims and depth of each batched circuit; the gates of circuit i are drawn
    lazily from their own seed so a single circuit can be rebuilt alone."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        while True:
            n = int(rng.integers(6, 17))
            dims = [int(x) for x in rng.integers(2, 6, size=n)]
            if math.prod(dims) <= cap:
                break
        depth = int(rng.integers(depth_lo, depth_hi + 1))
        specs.append(CircuitSpec(dims, depth, seed * 100003 + i))
    return specs


def served_dims(rng: np.random.Generator, lo: float = 1e3, hi: float = 1e8) -> List[int]:
    """Register whose size is close to a log-uniform target S in [lo, hi]."""
    while True:
        S = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi))
        p, dims, misses = 1, [], 0
        while misses < 8:
            d = int(rng.integers(2, 8))
            if p * d <= S:
                dims.append(d)
                p *= d
            else:
                misses += 1
        if p >= lo:
            return dims


@dataclass
class Request:
    rid: int
    arrival: float
    spec: CircuitSpec


def served_requests(qps: float, count: int, seed: int = SEEDS["served"], lo: float = 1e3,
                    hi: float = 1e8, depth_lo: int = 50, depth_hi: int = 500) -> List[Request]:
    """Poisson arrivals at rate ``qps`` (exponential inter-arrival gaps)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / qps)) if qps > 0 else 0.0
        dims = served_dims(rng, lo, hi)
        depth = int(rng.integers(depth_lo, depth_hi + 1))
        out.append(Request(i, t, CircuitSpec(dims, depth, seed * 100003 + i)))
    return out
