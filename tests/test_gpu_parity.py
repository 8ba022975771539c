"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle,
element by element on the same seeded inputs.

Tolerances (max-abs amplitude error): complex128 <= 1e-12, complex64 <= 2e-5
and additionally <= 1e-5 of the largest amplitude. Permutation gates and
amplitudes outside the controls must match bit for bit.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, gpu_values, max_abs, rand_monomial, rand_state, upload_chunks
from qd_inputs import Gate, circuits, clock, dft, haar, shift, states

pytestmark = pytest.mark.gpu

PRECISIONS = ["c128", "c64"]


def qd():
    import paper_2410_17876_amd as q
    return q


def new_state(dims, precision, psi=None):
    st = qd().State(dims, precision)
    if psi is not None:
        st.set_amplitudes(psi)
    return st


def expect(precision, psi):
    """What the device holds after uploading psi (FP32-rounded for c64)."""
    if precision == "c64":
        return psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64)
    return psi.copy()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_worked_example(precision):
    st = new_state([2, 3], precision)
    st.apply([1], dft(3))
    st.apply([0], shift(2, 1), [1], [2])
    got = st.amplitudes()
    want = np.zeros(6, dtype=np.complex128)
    want[[0, 2, 5]] = 1 / math.sqrt(3)
    assert_close(got, want, precision, "worked example")
    p = st.probabilities("host")
    assert np.max(np.abs(p - np.abs(want) ** 2)) < (1e-15 if precision == "c128" else 1e-7)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_plain_circuit(precision):
    dims, gates = circuits.plain()
    st = new_state(dims, precision)
    ref = oracle.zero_state(dims)
    for i, g in enumerate(gates):
        st.apply_gate(g)
        oracle.apply_gate(dims, ref, g)
        if precision == "c128":
            assert_close(st.amplitudes(), ref, precision, f"gate {i} ({g.kind})")
    assert_close(st.amplitudes(), ref, precision, "final")
    assert abs(st.norm() - oracle.norm(ref)) < (1e-13 if precision == "c128" else 1e-6)


CASES = [
    [3, 5, 7, 2, 3, 4, 5],            # D = 25200, odd radices everywhere
    [2] * 10 + [3] * 4,               # D = 82944
    [7, 7, 7, 5],                     # D = 1715, fewer classes than a workgroup
    [2] * 8 + [3] * 5 + [5, 7],       # D = 2.18e6, many tiles and a ragged tail
    [4, 6, 2, 7, 3, 2, 5],            # D = 10080
]


def random_gate(rng, dims):
    n = len(dims)
    kind = rng.integers(6)
    k = int(rng.integers(1, min(3, n) + 1))
    targets = [int(x) for x in rng.choice(n, k, replace=False)]
    M = math.prod(dims[t] for t in targets)
    while M > 343:
        targets = targets[:-1]
        M = math.prod(dims[t] for t in targets)
    rest = [q for q in range(n) if q not in targets]
    m = int(rng.integers(0, min(2, len(rest)) + 1))
    controls = [int(x) for x in rng.choice(rest, m, replace=False)] if m else []
    values = [int(rng.integers(dims[c])) for c in controls]
    if kind <= 2:
        U = haar(M, rng)
    elif kind == 3:
        U = rand_monomial(rng, M)
    elif kind == 4:
        U = np.diag(np.exp(2j * np.pi * rng.random(M)))
    else:
        U = dft(M)
    return Gate(tuple(targets), U, tuple(controls), tuple(values))


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_random_circuits(precision, case):
    dims = CASES[case]
    rng = np.random.default_rng(100 + case)
    D = math.prod(dims)
    psi0 = rand_state(rng, D)
    n_gates = 12 if D > 10**6 else 40
    gates = [random_gate(rng, dims) for _ in range(n_gates)]
    st = new_state(dims, precision, psi0)
    ref = expect(precision, psi0)
    for g in gates:
        st.apply_gate(g)
        oracle.apply_gate(dims, ref, g)
    assert_close(st.amplitudes(), ref, precision, f"dims {dims}")


def family_cases():
    # (dims, targets): class sizes M = 2..16 in registers, 18..343 through LDS.
    out = []
    for d in range(2, 8):
        out.append(([3, d, 2, 5, 4], [1]))
    for dims, t in (([2, 4, 3], [0, 1]), ([3, 3, 2], [1, 0]), ([2, 5, 3], [1, 0]), ([4, 3, 2, 2], [0, 1]),
                    ([2, 7, 3], [0, 1]), ([5, 3, 2], [1, 0]), ([4, 4, 3], [0, 1]), ([3, 6, 2], [0, 1]),
                    ([5, 5, 2, 3], [0, 1]), ([7, 7, 2], [1, 0]), ([5, 5, 5, 2], [0, 1, 2]),
                    ([7, 7, 7, 2], [2, 0, 1]), ([2, 3, 3, 2, 2], [1, 3, 2])):
        out.append((dims, t))
    return out


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("dims,targets", family_cases())
def test_dense_every_class_size(precision, dims, targets):
    rng = np.random.default_rng(sum(dims) * 31 + len(targets))
    dims = list(dims) + [3, 2, 5]  # more free qudits so there are many classes
    D = math.prod(dims)
    M = math.prod(dims[t] for t in targets)
    psi0 = rand_state(rng, D)
    U = haar(M, rng)
    for controls, values in (((), ()), ((len(dims) - 1,), (3,))):
        st = new_state(dims, precision, psi0)
        ref = expect(precision, psi0)
        st.apply(targets, U, controls, values)
        oracle.apply(dims, ref, targets, U, controls, values)
        got = st.amplitudes()
        assert_close(got, ref, precision, f"M={M} controls={controls}")
        if controls:
            s = np.cumprod([1] + dims[:-1])
            j = np.arange(D)
            off = ((j // s[controls[0]]) % dims[controls[0]]) != values[0]
            assert np.array_equal(got[off], expect(precision, psi0)[off]), "amplitudes outside the controls moved"


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("A", [1, 2, 3, 5, 8, 11, 16])
def test_monomial_active_counts(precision, A):
    rng = np.random.default_rng(A)
    # M = 16 (two ququads) with M - A identity columns left in place.
    dims = [3, 4, 2, 4, 5]
    targets = [1, 3]
    M = 16
    U = rand_monomial(rng, M, phases=True, fixed=M - A)
    # move the fixed columns to random places by conjugating with a permutation
    P = np.eye(M)[rng.permutation(M)]
    U = P @ U @ P.T
    info = qd().gate_info(dims, targets, U)
    assert info["kernel"] == "sweep_monomial"
    psi0 = rand_state(rng, math.prod(dims))
    st = new_state(dims, precision, psi0)
    ref = expect(precision, psi0)
    st.apply(targets, U, [4], [2])
    oracle.apply(dims, ref, targets, U, [4], [2])
    assert_close(st.amplitudes(), ref, precision, f"A={A}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_shift_bit_exact_and_closed_form(precision):
    dims = [3, 2, 5, 4, 2, 7, 3, 2, 3]
    D = math.prod(dims)
    s = np.cumprod([1] + dims[:-1])
    psi0 = states.labelled(0, D)
    j = np.arange(D)
    st = new_state(dims, precision, psi0)
    for t in range(len(dims)):
        st.apply([t], shift(dims[t], 1))
        dig = (j // s[t]) % dims[t]
        src = j - dig * s[t] + ((dig - 1) % dims[t]) * s[t]
        assert np.array_equal(st.amplitudes(), psi0[src]), f"X_+1 on q{t}"
        for _ in range(dims[t] - 1):
            st.apply([t], shift(dims[t], 1))
        assert np.array_equal(st.amplitudes(), psi0), f"X^d on q{t}"
    # controlled shifts against the oracle, bit for bit
    ref = psi0.copy()
    rng = np.random.default_rng(3)
    for _ in range(20):
        c, t = (int(x) for x in rng.choice(len(dims), 2, replace=False))
        v = int(rng.integers(dims[c]))
        st.apply([t], shift(dims[t], 1), [c], [v])
        oracle.apply(dims, ref, [t], shift(dims[t], 1), [c], [v])
    assert np.array_equal(st.amplitudes(), ref)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_dft_everywhere_uniform(precision):
    dims = [2, 3, 4, 5, 7, 6, 2, 3]
    D = math.prod(dims)
    st = new_state(dims, precision)
    for t in range(len(dims)):
        st.apply([t], dft(dims[t]))
    got = st.amplitudes()
    tol = 1e-14 if precision == "c128" else 1e-6 / math.sqrt(D) * 10
    assert max_abs(got, np.full(D, 1 / math.sqrt(D))) < tol


@pytest.mark.parametrize("precision", PRECISIONS)
def test_roundtrip_and_norm(precision):
    rng = np.random.default_rng(5)
    dims = [2, 3, 4, 5, 3, 2, 2, 3]
    D = math.prod(dims)
    psi0 = rand_state(rng, D)
    gates = [random_gate(rng, dims) for _ in range(30)]
    st = new_state(dims, precision, psi0)
    st.run(gates)
    n1 = st.norm()
    assert abs(n1 - 1.0) < (1e-13 if precision == "c128" else 1e-5)
    for g in reversed(gates):
        st.apply_gate(g.inverse())
    assert_close(st.amplitudes(), expect(precision, psi0), precision, "roundtrip")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_norm_probabilities_and_determinism(precision):
    rng = np.random.default_rng(6)
    dims = [2] * 12 + [3] * 6 + [5]
    D = math.prod(dims)
    psi0 = rand_state(rng, D) * 1.7
    st = new_state(dims, precision, psi0)
    held = expect(precision, psi0)
    n_gpu = st.norm()
    assert abs(n_gpu - oracle.norm(held)) <= 1e-13 * 1.7
    assert st.norm() == n_gpu  # fixed reduction order: bit-identical
    p = st.probabilities("host")
    p_ref = oracle.probabilities(held)
    assert np.max(np.abs(p - p_ref)) <= 4e-16 * np.max(p_ref)
    pd = st.probabilities("device").cpu().numpy()
    assert np.array_equal(pd, p)
    # a circuit run twice gives the same bits
    gates = [random_gate(rng, dims) for _ in range(15)]
    a = new_state(dims, precision, psi0).run(gates).amplitudes()
    b = new_state(dims, precision, psi0).run(gates).amplitudes()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_edge_cases(precision):
    rng = np.random.default_rng(7)
    # one qudit of every dim
    for d in range(2, 8):
        psi0 = rand_state(rng, d)
        U = haar(d, rng)
        st = new_state([d], precision, psi0)
        st.apply([0], U)
        ref = oracle.apply([d], expect(precision, psi0), [0], U)
        assert_close(st.amplitudes(), ref, precision, f"single qudit d={d}")
    # every qudit is a target or control: one class, no free segment
    dims = [3, 2, 5]
    psi0 = rand_state(rng, 30)
    for targets, controls, values in (([0, 1, 2], [], []), ([2, 0], [1], [1]), ([1], [0, 2], [2, 4])):
        M = math.prod(dims[t] for t in targets)
        U = haar(M, rng)
        st = new_state(dims, precision, psi0)
        st.apply(targets, U, controls, values)
        ref = oracle.apply(dims, expect(precision, psi0), targets, U, controls, values)
        assert_close(st.amplitudes(), ref, precision, f"no free qudits {targets} {controls}")
    # many controls (multi-controlled gate, Sec. 2.4)
    dims = [2, 3, 2, 2, 3, 2, 4, 2]
    psi0 = rand_state(rng, math.prod(dims))
    controls, values = [0, 1, 3, 4, 5, 7], [1, 2, 0, 1, 1, 0]
    U = haar(8, rng)
    st = new_state(dims, precision, psi0)
    st.apply([6, 2], U, controls, values)
    ref = oracle.apply(dims, expect(precision, psi0), [6, 2], U, controls, values)
    assert_close(st.amplitudes(), ref, precision, "multi-controlled")
    # identity gate is a no-op; basis reset
    st.apply([0], np.eye(2))
    assert_close(st.amplitudes(), ref, precision, "identity")
    st.reset(17)
    want = np.zeros(st.D, dtype=np.complex128)
    want[17] = 1
    assert np.array_equal(st.amplitudes(), want)


def test_errors_leave_state_untouched():
    q = qd()
    rng = np.random.default_rng(8)
    dims = [2, 3, 4]
    psi0 = rand_state(rng, 24)
    st = new_state(dims, "c128", psi0)
    for args in (([0, 0], np.eye(4), [], []), ([3], np.eye(2), [], []), ([0], np.eye(2), [1], [5]),
                 ([0], np.eye(2), [0], [0]), ([0, 1, 2, 0], np.eye(48), [], [])):
        with pytest.raises(q.QDError):
            st.apply(*args)
    assert np.array_equal(st.amplitudes(), psi0)
    with pytest.raises(q.QDError):
        st.reset(24)
    with pytest.raises(q.QDError) as e:
        q.State([2, 3], "c128", init=None).amplitudes(5, 2)
    assert e.value.code == -1


def test_64bit_index_path():
    # D = 2^31 takes the 64-bit decoder; check sampled outputs of single gates
    # against the oracle's sampled form on an index-labelled input (exact in FP32).
    import torch

    dims = [2] * 31
    D = 2**31
    st = qd().State(dims, "c64", init=None)
    upload_chunks(st, lambda s, c: states.labelled(s, c), chunk=1 << 24)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.integers(0, D, size=4000), [0, 1, D - 2, D - 1]])
    for g in (Gate((30,), shift(2)), Gate((0,), shift(2), (30,), (1,)), Gate((5, 29), rand_monomial(rng, 4, False))):
        st.apply_gate(g)
        want = oracle.apply_sampled(dims, g, idx, states.labelled_at)
        assert np.array_equal(gpu_values(st, idx), want)
        st.apply_gate(g.inverse())
    g = Gate((17, 3), haar(4, rng), (30,), (0,))
    st.apply_gate(g)
    want = oracle.apply_sampled(dims, g, idx, states.labelled_at)
    got = gpu_values(st, idx)
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))
    del st
    torch.cuda.empty_cache()


def test_state_on_side_stream():
    import torch

    rng = np.random.default_rng(10)
    dims = [3, 4, 2, 5, 2]
    psi0 = rand_state(rng, math.prod(dims))
    gates = [random_gate(rng, dims) for _ in range(20)]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        st = new_state(dims, "c128", psi0)
        st.run(gates)
        got = st.amplitudes()
    ref = oracle.run(dims, gates, psi0)
    assert_close(got, ref, "c128", "side stream")
