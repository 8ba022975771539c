"""Seeded synthetic inputs for mixed-radix qudit simulation.

This module is shared by the GPU library's tests and benchmark and by the CPU
oracle's tests. It only *produces inputs*: gate matrices, gate lists (circuits)
and initial statevectors. It holds none of the simulation arithmetic (no gate
application, no class enumeration, no reductions), so it can serve both sides
without coupling them.

Submodules:
  gates     standard qudit gates (generalized DFT, shift X_{+a}, clock Z) and
            Haar-random unitaries
  circuits  seeded gate-list generators for the workload configurations
  states    seeded initial statevectors (|0..0>, basis states, index-labelled
            states, chunked complex Gaussian states addressable by index)
"""
from .gates import Gate, dft, shift, clock, haar, dagger
from . import circuits, states

__all__ = ["Gate", "dft", "shift", "clock", "haar", "dagger", "circuits", "states"]
