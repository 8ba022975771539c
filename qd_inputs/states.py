"""Seeded initial statevectors.

Amplitude j belongs to basis state |j>, with q_0 the least significant qudit
(paper Sec. 2). States are complex128 numpy arrays unless noted.

The complex Gaussian state is defined chunk by chunk so that any amplitude can
be produced without materialising the whole vector: chunk c (CHUNK amplitudes,
the last one possibly shorter) holds the standard normals drawn by
``numpy.random.default_rng([seed, c])`` in (re, im) interleaved order; the
normalised state is those values times 1/sqrt(sum of squares), the sum taken in
FP64 per chunk and combined with ``math.fsum``.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Optional

import numpy as np

CHUNK = 1 << 20


def dim(dims) -> int:
    return int(math.prod(int(d) for d in dims))


def zero_state(dims) -> np.ndarray:
    psi = np.zeros(dim(dims), dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis_state(dims, j: int) -> np.ndarray:
    psi = np.zeros(dim(dims), dtype=np.complex128)
    psi[j] = 1.0
    return psi


def labelled(start: int, count: int) -> np.ndarray:
    """psi[j] = (j mod 2^20) + i (j >> 20): every value is an integer that FP32
    holds exactly for j < 2^44, so moves of amplitudes can be checked bit-exactly
    in both precisions."""
    j = np.arange(start, start + count, dtype=np.int64)
    return (j & 0xFFFFF).astype(np.float64) + 1j * (j >> 20).astype(np.float64)


def labelled_at(idx) -> np.ndarray:
    """The index-labelled state's values at arbitrary indices."""
    j = np.asarray(idx, dtype=np.int64)
    return (j & 0xFFFFF).astype(np.float64) + 1j * (j >> 20).astype(np.float64)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class GaussianState:
    """Normalised complex Gaussian state of dimension D, addressable by index."""

    def __init__(self, D: int, seed: int, chunk: int = CHUNK):
        self.D = int(D)
        self.seed = int(seed)
        self.chunk = int(chunk)
        self.nchunks = (self.D + self.chunk - 1) // self.chunk
        self._scale: Optional[float] = None
        self._cache: "dict[int, np.ndarray]" = {}
        self.cache_chunks = 0  # chunks kept by values(); 0 = none

    def _raw(self, c: int) -> np.ndarray:
        n = min(self.chunk, self.D - c * self.chunk)
        rng = np.random.default_rng([self.seed, c])
        return rng.standard_normal(2 * n)  # interleaved re, im

    def _sumsq(self, c: int) -> float:
        g = self._raw(c)
        return float(np.dot(g, g))

    @property
    def scale(self) -> float:
        if self._scale is None:
            with ThreadPoolExecutor(_threads()) as ex:
                parts = list(ex.map(self._sumsq, range(self.nchunks)))
            self._scale = 1.0 / math.sqrt(math.fsum(parts))
        return self._scale

    def chunk_values(self, c: int, scale: Optional[float] = None) -> np.ndarray:
        """Interleaved FP64 (re, im) values of chunk c, normalised."""
        s = self.scale if scale is None else scale
        g = self._raw(c)
        g *= s
        return g

    def values(self, idx: np.ndarray) -> np.ndarray:
        """complex128 amplitudes at the given indices."""
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty(idx.shape, dtype=np.complex128)
        flat = idx.ravel()
        res = out.ravel()
        ch = flat // self.chunk
        s = self.scale
        for c in np.unique(ch):
            c = int(c)
            sel = np.nonzero(ch == c)[0]
            v = self._cache.get(c)
            if v is None:
                v = self.chunk_values(c, s).view(np.complex128)
                if len(self._cache) < self.cache_chunks:
                    self._cache[c] = v
            res[sel] = v[flat[sel] - c * self.chunk]
        return out

    def fill(self, sink: Callable[[int, np.ndarray], None], window: int = 0) -> None:
        """Produce every chunk (normalised, interleaved FP64) and hand it to
        ``sink(start_index, values)`` in ascending order."""
        s = self.scale
        nt = _threads()
        window = window or 2 * nt
        with ThreadPoolExecutor(nt) as ex:
            futs = {}
            nxt = 0
            for c in range(self.nchunks):
                while nxt < self.nchunks and nxt < c + window:
                    futs[nxt] = ex.submit(self.chunk_values, nxt, s)
                    nxt += 1
                sink(c * self.chunk, futs.pop(c).result())

    def full(self) -> np.ndarray:
        """The whole normalised state as complex128 (D * 16 bytes of host memory)."""
        out = np.empty(2 * self.D, dtype=np.float64)

        def sink(start, vals):
            out[2 * start: 2 * start + vals.size] = vals

        self.fill(sink)
        return out.view(np.complex128)
