"""Gate matrices and the gate record used by every gate list.

Conventions (shared by the library and the oracle, stated once here):
  * A gate acts on an ordered list of target qudits ``targets = [t_0, ..., t_{k-1}]``.
    Its matrix ``U`` is M x M with M = prod d_{t_l}; the local index of a basis
    state is a = sum_l a_l * prod_{l' < l} d_{t_l'}, i.e. the FIRST listed target
    is the least significant local digit (mirroring q_0 being the least
    significant qudit of the register, paper Sec. 2).
  * Column a of U is the image of local basis state |a> (paper Sec. 2.3: the
    basis state with the target in |j> is transformed by the j-th column), so the
    new amplitudes are psi' = U psi on every class. U is stored row-major,
    U[out, in].
  * ``controls``/``values``: the gate acts only on basis states whose control
    qudit c_l holds value v_l (paper Sec. 2.4); elsewhere it is the identity.

The paper names the generalized Hadamard, the generalized Z and the shift
X_{+a}^d without giving matrices for d > 2 (Sec. 2.1-2.3); the readings used
here are the standard Weyl-Heisenberg ones: F_d[j, k] = w^{jk}/sqrt(d),
Z_d = diag(w^j), X_{+a}|j> = |(j + a) mod d>, w = exp(2 pi i / d).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


def dft(d: int) -> np.ndarray:
    """Generalized Hadamard (quantum Fourier transform on one qudit)."""
    j = np.arange(d)
    return np.exp(2j * np.pi * np.outer(j, j) / d) / np.sqrt(d)


def shift(d: int, a: int = 1) -> np.ndarray:
    """Generalized NOT X_{+a}^d: |j> -> |(j + a) mod d> (paper Sec. 2.2)."""
    X = np.zeros((d, d), dtype=np.complex128)
    for j in range(d):
        X[(j + a) % d, j] = 1.0
    return X


def clock(d: int) -> np.ndarray:
    """Generalized Z: diag(w^j), w = exp(2 pi i / d) (a phase gate, paper Sec. 2.1)."""
    return np.diag(np.exp(2j * np.pi * np.arange(d) / d))


def haar(M: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random M x M unitary.

    QR of a complex Ginibre matrix Z = (A + iB)/sqrt(2) with the phases of R's
    diagonal moved into Q (Mezzadri, "How to generate random matrices from the
    classical compact groups", Notices AMS 54(5), 2007). Without the phase fix
    the result is unitary but not Haar distributed.
    """
    Z = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    ph = np.diagonal(R) / np.abs(np.diagonal(R))
    return Q * ph[None, :]


def dagger(U: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(U.conj().T)


@dataclass
class Gate:
    """One gate of a gate list.

    ``kind`` is a descriptive label only ("haar1", "haar2", "haar3", "dft",
    "x", "z", "cx", ...); neither the library nor the oracle reads it.
    """

    targets: Tuple[int, ...]
    U: np.ndarray
    controls: Tuple[int, ...] = ()
    values: Tuple[int, ...] = ()
    kind: str = "u"

    def __post_init__(self):
        self.targets = tuple(int(t) for t in self.targets)
        self.controls = tuple(int(c) for c in self.controls)
        self.values = tuple(int(v) for v in self.values)
        self.U = np.ascontiguousarray(np.asarray(self.U, dtype=np.complex128))

    @property
    def M(self) -> int:
        return int(self.U.shape[0])

    def inverse(self) -> "Gate":
        return Gate(self.targets, dagger(self.U), self.controls, self.values, self.kind + "^-1")
