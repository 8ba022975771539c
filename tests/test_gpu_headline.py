"""The benchmark's headline path checked against the FP64 oracle.

The benchmark times qd_apply_circuit with LDS-staged fusion, a 256-gate
commuting look-ahead and the library's default tiles on the 500-gate circuit of
the large workload (a 2-qudit Haar unitary w.p. 0.1, else the basic mix) from a
normalised complex Gaussian state. Here the same options run:

  * on the scaled-down register 2^10 x 3^6 x 4^2 (D = 1.19e7), where the oracle
    holds the whole state: every amplitude is compared with the oracle's result
    of the 500 gates in the given order (complex128 <= 1e-12; complex64 <= 2e-5
    and <= 1e-5 x max|psi|), and bitwise with one sweep per gate in the planned
    order (Sec. 2.3: the passes apply the same per-class arithmetic);
  * on the full register 2^14 x 3^8 x 4^2 (D = 1.72e9), where the whole fused
    state must equal, bit for bit, one sweep per gate in the planned order
    (whose single gates are checked against the oracle at this size in
    test_gpu_large.py), and the inverse circuit through the same path must
    return the input on sampled amplitudes;
  * on registers with D >= 2^31, where the fused kernel takes 64-bit indices and
    run offsets: permutation passes must match the oracle's sampled form bit
    for bit on an index-labelled input, and dense passes within the tolerances.
"""
import math
import os

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, gpu_values, upload_chunks
from qd_inputs import Gate, circuits, haar, shift, states

pytestmark = pytest.mark.gpu

LOOKAHEAD = 256
SMALL_DIMS = [2] * 10 + [3] * 6 + [4] * 2


def qd():
    import paper_2410_17876_amd as q
    return q


def round32(v):
    return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def small_case():
    """Input, gates and the oracle's results of the 500 gates on the small
    register: from the FP64 input (for complex128) and from that input rounded
    once to FP32 (for complex64, whose state starts from the rounded values)."""
    dims, gates = circuits.large(dims=SMALL_DIMS)
    D = math.prod(dims)
    psi0 = states.GaussianState(D, seed=circuits.SEEDS["large"]).full()
    print(f"[headline small] oracle: {len(gates)} gates on D={D}", flush=True)
    with oracle.threads(min(16, os.cpu_count() or 1)):
        ref = {"c128": oracle.run(dims, gates, psi0), "c64": oracle.run(dims, gates, round32(psi0))}
    return dims, gates, psi0, ref


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_headline_path_small_register_vs_oracle(small_case, precision):
    dims, gates, psi0, refs = small_case
    ref = refs[precision]
    print(f"[headline small {precision}] qd_apply_circuit reorder={LOOKAHEAD}, default tiles", flush=True)
    gl = qd().GateList(gates)
    passes, order = qd().circuit_plan(dims, gl, precision, reorder=LOOKAHEAD, with_order=True)
    a = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    info = a.run_circuit(gl, reorder=LOOKAHEAD)
    assert info["passes"] == len(passes)
    assert info["fused_passes"] >= 1
    got = a.amplitudes()
    a.close()
    err = float(np.max(np.abs(got - ref)))
    print(f"[headline small {precision}] {len(passes)} passes; max-abs error vs oracle {err:.3e}, "
          f"relative {err / float(np.max(np.abs(ref))):.3e}", flush=True)
    assert_close(got, ref, precision, f"headline path, 500 gates, {precision}")
    b = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    b.run([gates[i] for i in order])
    assert np.array_equal(got, b.amplitudes()), "fused look-ahead differs from one sweep per gate in planned order"
    b.close()


@pytest.fixture(scope="module")
def large_gen():
    G = states.GaussianState(math.prod(circuits.LARGE_DIMS), seed=circuits.SEEDS["large"])
    G.cache_chunks = 64
    return G


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_headline_path_full_size(large_gen, precision):
    import torch

    dims, gates = circuits.large()
    D = math.prod(dims)
    gl = qd().GateList(gates)
    passes, order = qd().circuit_plan(dims, gl, precision, reorder=LOOKAHEAD, with_order=True)
    print(f"[headline full {precision}] D={D}, {len(passes)} passes", flush=True)
    a = qd().State(dims, precision, init=None)
    large_gen.fill(lambda start, vals: a.set_interleaved(vals, start))
    b = qd().State(dims, precision, init=None)
    b.buffer.copy_(a.buffer)
    a.run_circuit(gl, reorder=LOOKAHEAD)
    b.run([gates[i] for i in order])
    torch.cuda.synchronize()
    same = bool(torch.equal(a.buffer, b.buffer))
    print(f"[headline full {precision}] fused == one sweep per gate (planned order): {same}", flush=True)
    assert same, "fused look-ahead differs from one sweep per gate in the planned order"
    b.close()
    del b
    torch.cuda.empty_cache()
    nrm = a.norm()
    assert abs(nrm - 1.0) < (1e-12 if precision == "c128" else 1e-5)
    inv = qd().GateList([g.inverse() for g in reversed(gates)])
    a.run_circuit(inv, reorder=LOOKAHEAD)
    rng = np.random.default_rng(44)
    chunks = rng.choice(large_gen.nchunks, 12, replace=False)
    idx = np.concatenate([int(c) * large_gen.chunk + rng.integers(0, min(large_gen.chunk, D - int(c) * large_gen.chunk),
                                                                  size=256) for c in chunks] + [np.array([0, D - 1])])
    want = large_gen.values(idx)
    if precision == "c64":
        want = round32(want)
    got = gpu_values(a, idx)
    err = float(np.max(np.abs(got - want)))
    print(f"[headline full {precision}] 1000-gate look-ahead roundtrip max-abs error {err:.3e}", flush=True)
    assert_close(got, want, precision, f"look-ahead roundtrip {precision}")
    a.close()
    del a
    torch.cuda.empty_cache()


def sampled_through(dims, gates, idx, inputs):
    """Oracle values at idx after gates[0..n-1] applied to the input given by
    inputs(idx): each gate's sampled form takes its inputs from the previous
    gate's sampled form (fan-in M per gate, so keep the lists short)."""
    f = inputs
    for g in gates:
        f = (lambda g, prev: (lambda ix: oracle.apply_sampled(dims, g, ix, prev)))(g, f)
    return f(np.asarray(idx, dtype=np.int64))


def labelled_scaled_at(idx):
    # index-labelled values times 2^-40: exact in FP32, magnitudes below 2^-20
    return states.labelled_at(idx) * 2.0 ** -40


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_fused_64bit_indices(precision):
    import torch

    dims = [2] * 31  # D = 2^31: 64-bit indices and run offsets in the fused kernel
    D = 2**31
    st = qd().State(dims, precision, init=None)
    print(f"[fused 64-bit {precision}] D={D}: uploading the labelled state", flush=True)
    upload_chunks(st, lambda s, c: states.labelled(s, c) * 2.0 ** -40, chunk=1 << 24)
    rng = np.random.default_rng(31)
    idx = np.concatenate([rng.integers(0, D, size=3000), [0, 1, 2**30, 2**31 - 2, 2**31 - 1]])
    P4 = np.eye(4)[[2, 0, 3, 1]].T  # a permutation without phases
    perm_pass = [Gate((0,), shift(2)), Gate((30,), shift(2)), Gate((1,), shift(2), (29,), (1,)),
                 Gate((3, 30), P4), Gate((2,), shift(2), (28, 0), (0, 1)), Gate((29,), shift(2), (4,), (1,))]
    info = st.run_circuit(perm_pass)
    print(f"[fused 64-bit {precision}] permutation pass: {info}", flush=True)
    assert info["fused_passes"] == info["passes"] == 1
    want = sampled_through(dims, perm_pass, idx, labelled_scaled_at)
    assert np.array_equal(gpu_values(st, idx), want)
    inv = [g.inverse() for g in reversed(perm_pass)]
    st.run_circuit(inv)
    assert np.array_equal(gpu_values(st, idx), labelled_scaled_at(idx))
    dense_pass = [Gate((30,), haar(2, rng)), Gate((0, 5), haar(4, rng)), Gate((2,), haar(2, rng), (29,), (1,)),
                  Gate((1,), haar(2, rng))]
    info = st.run_circuit(dense_pass)
    print(f"[fused 64-bit {precision}] dense pass: {info}", flush=True)
    assert info["fused_passes"] == info["passes"] == 1
    want = sampled_through(dims, dense_pass, idx, labelled_scaled_at)
    assert_close(gpu_values(st, idx), want, precision, "dense pass, 64-bit indices")
    st.run_circuit([g.inverse() for g in reversed(dense_pass)])
    assert_close(gpu_values(st, idx), labelled_scaled_at(idx), precision, "dense pass and inverse, 64-bit indices")
    st.close()
    del st
    torch.cuda.empty_cache()
