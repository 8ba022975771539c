"""Sparse form of the oracle (test infrastructure only, like the rest of oracle/).

The paper's sparse variant (Sec. 3, GHZ experiments) keeps only the nonzero
amplitudes, in a map from basis index to amplitude. A gate (Sec. 2.3, 2.4):
the entries whose controls hold are grouped by class (their index with the
target digits set to 0, the local index from the target digits, first target
least significant); every class with a present member gets y = U x with its
absent members 0, summed in ascending column order with textbook complex
products; the nonzero results replace the class; entries whose controls fail
are kept. Plain Python over a dict: slow, and obviously that.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np


def zero_state(dims: Sequence[int]) -> Dict[int, complex]:
    return {0: 1.0 + 0.0j}


def apply(dims, state: Dict[int, complex], targets, U, controls=(), values=()) -> Dict[int, complex]:
    """The new sparse state (a new dict) after one gate."""
    s = [math.prod(dims[:i]) for i in range(len(dims))]
    dig = lambda j, q: (j // s[q]) % dims[q]
    U = np.asarray(U, dtype=np.complex128)
    M = U.shape[0]
    off = []
    for a in range(M):
        o, r = 0, a
        for t in targets:
            o += (r % dims[t]) * s[t]
            r //= dims[t]
        off.append(o)
    out: Dict[int, complex] = {}
    classes: Dict[int, Dict[int, complex]] = {}
    for j, amp in state.items():
        if all(dig(j, c) == v for c, v in zip(controls, values)):
            a, w, base = 0, 1, j
            for t in targets:
                a += dig(j, t) * w
                w *= dims[t]
                base -= dig(j, t) * s[t]
            classes.setdefault(base, {})[a] = amp
        else:
            out[j] = amp
    for base, xs in classes.items():
        for r in range(M):
            yr, yi = 0.0, 0.0
            for a in range(M):
                if a in xs:
                    ur, ui = U[r, a].real, U[r, a].imag
                    xr, xi = xs[a].real, xs[a].imag
                    yr = yr + (ur * xr - ui * xi)
                    yi = yi + (ur * xi + ui * xr)
            if yr != 0.0 or yi != 0.0:
                out[base + off[r]] = complex(yr, yi)
    return out


def run(dims, gates, state=None) -> Dict[int, complex]:
    st = zero_state(dims) if state is None else dict(state)
    for g in gates:
        st = apply(dims, st, g.targets, g.U, g.controls, g.values)
    return st
