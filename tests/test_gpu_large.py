"""Parity at the benchmark's full size: the register 2^14 x 3^8 x 4^2
(D = 1.72e9 amplitudes, 27.5 GB in complex128), one sweep per gate
(qd_apply_gate). The fused look-ahead passes the benchmark times are checked at
this size in test_gpu_headline.py.

The oracle cannot hold this state, so single gates are checked on sampled
outputs: each sampled output amplitude depends on the M inputs of its class,
which the oracle's sampled form takes straight from the seeded input generator
(never from the GPU). After each gate its inverse returns the state to the
input (checked on the same samples) before the next gate. The whole 500-gate
circuit is then checked through properties that hold at any size: the norm is
kept, and the circuit followed by its inverse returns the input.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, gpu_values
from qd_inputs import Gate, circuits, clock, dft, haar, shift, states

pytestmark = pytest.mark.gpu

DIMS = circuits.LARGE_DIMS
D = math.prod(DIMS)


def round32(v):
    return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)


def sample_indices(rng, G, n_chunks=12, per_chunk=256):
    chunks = rng.choice(G.nchunks, n_chunks, replace=False)
    idx = [int(c) * G.chunk + rng.integers(0, min(G.chunk, D - int(c) * G.chunk), size=per_chunk)
           for c in chunks]
    return np.concatenate(idx + [np.array([0, 1, D - 2, D - 1])])


def gate_selection(rng):
    d = DIMS
    out = [Gate((0,), haar(2, rng)), Gate((5,), haar(2, rng)), Gate((13,), haar(2, rng)),
           Gate((14,), haar(3, rng)), Gate((21,), dft(3)), Gate((23,), haar(4, rng)), Gate((22,), clock(4)),
           Gate((0,), shift(2)), Gate((17,), shift(3)), Gate((0,), shift(2), (23,), (3,)),
           Gate((20,), shift(3), (1,), (0,)), Gate((0, 23), haar(8, rng)), Gate((14, 3), haar(6, rng)),
           Gate((22, 23), haar(16, rng)), Gate((2, 15, 22), haar(24, rng))]
    _, bench = circuits.large()
    return out + bench[:6]


@pytest.fixture(scope="module")
def gen():
    G = states.GaussianState(D, seed=circuits.SEEDS["large"])
    G.cache_chunks = 160
    return G


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_single_gates_sampled(gen, precision):
    import torch
    import paper_2410_17876_amd as qd

    st = qd.State(DIMS, precision, init=None)
    gen.fill(lambda start, vals: st.set_interleaved(vals, start))
    rng = np.random.default_rng(42)
    idx = sample_indices(rng, gen)
    inp = gen.values if precision == "c128" else (lambda ix: round32(gen.values(ix)))
    for g in gate_selection(rng):
        print(f"[large {precision}] gate targets={g.targets} controls={g.controls} kind={g.kind}", flush=True)
        st.apply_gate(g)
        want = oracle.apply_sampled(DIMS, g, idx, inp)
        assert_close(gpu_values(st, idx), want, precision, f"{g.kind} on {g.targets}")
        st.apply_gate(g.inverse())
        assert_close(gpu_values(st, idx), inp(idx), precision, f"inverse of {g.kind} on {g.targets}")
    st.close()
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_full_circuit_roundtrip(gen, precision):
    import torch
    import paper_2410_17876_amd as qd

    _, gates = circuits.large()
    st = qd.State(DIMS, precision, init=None)
    gen.fill(lambda start, vals: st.set_interleaved(vals, start))
    st.run(gates)
    nrm = st.norm()
    print(f"[large {precision}] norm after 500 gates: {nrm!r}", flush=True)
    assert abs(nrm - 1.0) < (1e-12 if precision == "c128" else 1e-5)
    for g in reversed(gates):
        st.apply_gate(g.inverse())
    rng = np.random.default_rng(43)
    idx = sample_indices(rng, gen)
    want = gen.values(idx) if precision == "c128" else round32(gen.values(idx))
    got = gpu_values(st, idx)
    err = float(np.max(np.abs(got - want)))
    print(f"[large {precision}] 1000-gate roundtrip max-abs error {err:.3e}", flush=True)
    assert_close(got, want, precision, f"1000-gate roundtrip {precision}")
    st.close()
    del st
    torch.cuda.empty_cache()
