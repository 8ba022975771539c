"""LDS-staged fusion (qd_apply_circuit): the fused result must equal the
one-sweep-per-gate result bit for bit (same per-class arithmetic; in the given
order, or with look-ahead in the planned order) and the FP64 oracle within the
tolerances."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, rand_monomial, rand_state
from qd_inputs import Gate, circuits, clock, dft, haar, shift, states

pytestmark = pytest.mark.gpu


def qd():
    import paper_2410_17876_amd as q
    return q


def mixed_gates(rng, dims, count, max_m=16):
    n = len(dims)
    out = []
    while len(out) < count:
        k = int(rng.integers(1, min(3, n) + 1))
        t = [int(x) for x in rng.choice(n, k, replace=False)]
        M = math.prod(dims[x] for x in t)
        if M > max_m:
            continue
        rest = [q for q in range(n) if q not in t]
        m = int(rng.integers(0, min(3, len(rest)) + 1))
        c = [int(x) for x in rng.choice(rest, m, replace=False)] if m else []
        v = [int(rng.integers(dims[x])) for x in c]
        kind = int(rng.integers(5))
        U = haar(M, rng) if kind < 2 else (rand_monomial(rng, M) if kind == 2 else
                                           (np.diag(np.exp(2j * np.pi * rng.random(M))) if kind == 3 else
                                            (np.eye(M) if rng.random() < 0.2 else dft(M))))
        out.append(Gate(tuple(t), U, tuple(c), tuple(v)))
    return out


CASES = [
    ([2] * 8 + [3] * 4 + [4, 5], 4096, 64),     # D = 1.66e6
    ([3, 5, 7, 2, 3, 4, 5, 2, 2], 4096, 64),   # odd radices; low block 105
    ([2] * 18, 1024, 32),                      # small tiles
    ([4, 3, 2, 5, 7, 3, 2, 2, 3], 8192, 128),  # big tile
    ([2, 3, 2, 2, 3, 5], 4096, 64),            # D = 720 <= tile: the whole circuit in one tile
]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_equals_sequential_and_oracle(precision, case):
    dims, tile, run = CASES[case]
    if precision == "c64":
        tile *= 2
    rng = np.random.default_rng(500 + case)
    D = math.prod(dims)
    psi0 = rand_state(rng, D)
    gates = mixed_gates(rng, dims, 60)
    a = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    info = a.run_circuit(gates, fuse=True, tile_amps=tile, min_run=run)
    assert info["fused_passes"] >= 1
    b = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    b.run_circuit(gates, fuse=False)
    c = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    c.run(gates)
    ga, gb, gc = a.amplitudes(), b.amplitudes(), c.amplitudes()
    assert np.array_equal(gb, gc)
    assert np.array_equal(ga, gc), f"fused differs from sequential: {np.max(np.abs(ga - gc)):.3e}"
    ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                   1j * psi0.imag.astype(np.float32).astype(np.float64))
    for g in gates:
        oracle.apply_gate(dims, ref, g)
    assert_close(ga, ref, precision, f"fused {dims}")


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_reordered_passes_equal_planned_order_and_oracle(precision, case):
    # With look-ahead the passes apply commuting gates out of the given order:
    # bitwise the one-by-one result in the planned order, and the oracle's
    # result in the given order within the tolerances.
    dims, tile, run = CASES[case]
    if precision == "c64":
        tile *= 2
    rng = np.random.default_rng(700 + case)
    psi0 = rand_state(rng, math.prod(dims))
    gates = mixed_gates(rng, dims, 80)
    passes, order = qd().circuit_plan(dims, gates, precision, tile_amps=tile, min_run=run, reorder=64,
                                      with_order=True)
    a = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    info = a.run_circuit(gates, tile_amps=tile, min_run=run, reorder=64)
    assert info["passes"] == len(passes)
    c = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    c.run([gates[i] for i in order])
    assert np.array_equal(a.amplitudes(), c.amplitudes())
    ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                   1j * psi0.imag.astype(np.float32).astype(np.float64))
    for g in gates:
        oracle.apply_gate(dims, ref, g)
    assert_close(a.amplitudes(), ref, precision, f"reordered {dims}")


def chain_gates(rng, dims):
    # runs of dense gates on the same targets (M = 2, 3, 4; a run longer than one
    # chain descriptor holds; controls inside and outside the tile) with
    # commuting gates on other qudits in between
    out = []
    runs = [((0,), (), ()), ((2,), (), ()), ((1,), (5,), (1,)), ((3,), (0,), (1,)), ((0, 4), (), ()),
            ((7,), (), ())]
    for targets, controls, values in runs:
        M = math.prod(dims[t] for t in targets)
        for j in range(int(rng.integers(3, 7)) if targets != (0,) else 20):
            out.append(Gate(targets, haar(M, rng), controls, values))
            if j % 3 == 2:  # a gate elsewhere: dense, monomial or diagonal, on qudits the run does not use
                q = 6 if 6 not in targets else 8
                out.append(Gate((q,), [haar(dims[q], rng), shift(dims[q]), clock(dims[q])][j % 3 - 2 + int(rng.integers(3))]))
    return out


def group_gates(rng, dims, count):
    # mostly uncontrolled 1-qudit gates of every category on qubits and qutrits
    # (group candidates), broken up by controlled and 2-qudit gates
    n, out = len(dims), []
    small = [q for q in range(n) if dims[q] <= 3]
    while len(out) < count:
        r = rng.random()
        if r < 0.8:
            q = int(rng.choice(small))
            d = dims[q]
            kind = int(rng.integers(6))
            U = [haar(d, rng), dft(d), shift(d, int(rng.integers(1, d)) if d > 1 else 0), clock(d),
                 rand_monomial(rng, d), np.diag(np.where(rng.random(d) < 0.5, 1.0, np.exp(2j * np.pi * rng.random(d))))][kind]
            out.append(Gate((q,), U))
        elif r < 0.9:
            c, t = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(Gate((t,), haar(dims[t], rng), (c,), (int(rng.integers(dims[c])),)))
        else:
            a, b = (int(x) for x in rng.choice(small, 2, replace=False))
            out.append(Gate((a, b), haar(dims[a] * dims[b], rng)))
    return out


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("reorder", [0, 64])
def test_groups_bitwise(precision, reorder):
    dims = [2, 3, 2, 2, 3, 4, 2, 3, 2, 5, 2]
    rng = np.random.default_rng(41 + reorder)
    psi0 = rand_state(rng, math.prod(dims))
    gates = group_gates(rng, dims, 150)
    tile = 2048 if precision == "c128" else 4096
    passes, order = qd().circuit_plan(dims, gates, precision, tile_amps=tile, min_run=16, reorder=reorder,
                                      with_order=True)
    a = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    a.run_circuit(gates, tile_amps=tile, min_run=16, reorder=reorder)
    c = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    c.run([gates[i] for i in order])
    assert np.array_equal(a.amplitudes(), c.amplitudes())
    ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                   1j * psi0.imag.astype(np.float32).astype(np.float64))
    for g in gates:
        oracle.apply_gate(dims, ref, g)
    assert_close(a.amplitudes(), ref, precision, f"groups, reorder {reorder}")


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_dense_chains_bitwise(precision):
    dims = [2, 3, 3, 4, 2, 2, 3, 2, 5, 2, 3]
    rng = np.random.default_rng(31)
    psi0 = rand_state(rng, math.prod(dims))
    gates = chain_gates(rng, dims)
    tile = 2048 if precision == "c128" else 4096
    # in order: adjacent same-target gates form chains
    a = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    a.run_circuit(gates, tile_amps=tile, min_run=32)
    c = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    c.run(gates)
    assert np.array_equal(a.amplitudes(), c.amplitudes())
    # look-ahead: the runs are gathered across the gates in between
    passes, order = qd().circuit_plan(dims, gates, precision, tile_amps=tile, min_run=32, reorder=64, with_order=True)
    b = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    b.run_circuit(gates, tile_amps=tile, min_run=32, reorder=64)
    d = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    d.run([gates[i] for i in order])
    assert np.array_equal(b.amplitudes(), d.amplitudes())
    ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                   1j * psi0.imag.astype(np.float32).astype(np.float64))
    for g in gates:
        oracle.apply_gate(dims, ref, g)
    assert_close(a.amplitudes(), ref, precision, "chains in order")
    assert_close(b.amplitudes(), ref, precision, "chains with look-ahead")


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_plain_circuit_in_one_launch(precision):
    dims, gates = circuits.plain()
    st = qd().State(dims, precision)
    info = st.run_circuit(gates)
    assert info["passes"] == info["fused_passes"] == 1
    assert_close(st.amplitudes(), oracle.run(dims, gates), precision, "plain circuit, one launch")


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_fused_bit_exact_moves(precision):
    # permutations inside tiles: X^d on every qudit returns the labelled input bit for bit
    dims = [3, 2, 5, 4, 2, 7, 3, 2]
    psi0 = states.labelled(0, math.prod(dims))
    gates = [Gate((t,), shift(dims[t])) for t in range(len(dims)) for _ in range(dims[t])]
    st = qd().State(dims, precision, init=None).set_amplitudes(psi0)
    st.run_circuit(gates, tile_amps=512, min_run=32)
    assert np.array_equal(st.amplitudes(), psi0)


def test_large_tiles_and_errors():
    q = qd()
    rng = np.random.default_rng(9)
    dims = [2] * 16 + [3, 3]
    gates = mixed_gates(rng, dims, 40)
    psi0 = rand_state(rng, math.prod(dims))
    ref = q.State(dims, "c64", init=None).set_amplitudes(psi0)
    ref.run(gates)
    big = q.State(dims, "c64", init=None).set_amplitudes(psi0)
    big.run_circuit(gates, tile_amps=16384, min_run=128)   # 128 KB of LDS per workgroup
    assert np.array_equal(big.amplitudes(), ref.amplitudes())
    with pytest.raises(q.QDError):
        big.run_circuit(gates, tile_amps=65536)
    bad = list(gates) + [Gate((0, 0), np.eye(4))]
    before = big.amplitudes()
    with pytest.raises(q.QDError):
        big.run_circuit(bad)
    assert np.array_equal(big.amplitudes(), before)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_dense_pairs_bitwise(precision):
    # Consecutive uncontrolled dense gates with classes of at most 4 amplitudes
    # run two at a time in registers; every (M1, M2) in {2,3,4}^2 occurs, plus a
    # 2-qubit gate followed by a 1-qudit gate. Fused, batched (device-decoded
    # bases) and sequential results must agree bit for bit.
    q = qd()
    dims = [2, 3, 4, 2, 3, 2, 4, 2, 2, 3]
    rng = np.random.default_rng(77)
    by_dim = {d: [i for i, x in enumerate(dims) if x == d] for d in (2, 3, 4)}
    gates = []
    for _ in range(3):
        for m1 in (2, 3, 4):
            for m2 in (2, 3, 4):
                q1 = int(rng.choice(by_dim[m1]))
                q2 = int(rng.choice([x for x in by_dim[m2] if x != q1]))
                gates += [Gate((q1,), haar(m1, rng)), Gate((q2,), haar(m2, rng))]
    gates += [Gate((0, 3), haar(4, rng)), Gate((1,), haar(3, rng)), Gate((4,), dft(3)), Gate((2,), dft(4))]
    psi0 = rand_state(rng, math.prod(dims))
    tile = 4096 if precision == "c128" else 8192
    fused = q.State(dims, precision, init=None).set_amplitudes(psi0)
    fused.run_circuit(gates, tile_amps=tile, min_run=64)
    seq = q.State(dims, precision, init=None).set_amplitudes(psi0)
    seq.run(gates)
    assert np.array_equal(fused.amplitudes(), seq.amplitudes())
    runner = q.batch.BatchRunner([dims], precision)
    runner.states[0].set_amplitudes(psi0)
    runner.run([gates], tile_amps=tile, min_run=64)
    assert np.array_equal(runner.states[0].amplitudes(), seq.amplitudes())
    runner.close()
    ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                   1j * psi0.imag.astype(np.float32).astype(np.float64))
    for g in gates:
        oracle.apply_gate(dims, ref, g)
    assert_close(fused.amplitudes(), ref, precision, "dense pairs")


def test_long_passes_with_large_tiles():
    # 300 gates on the low qubits with 16384-amplitude tiles: passes are cut by
    # the bound on their device data, and the result is the sequential one
    q = qd()
    rng = np.random.default_rng(8)
    dims = [2] * 20
    gates = [Gate((int(rng.integers(0, 15)),), haar(2, rng)) for _ in range(300)]
    psi0 = rand_state(rng, math.prod(dims))
    a = q.State(dims, "c64", init=None).set_amplitudes(psi0)
    info = a.run_circuit(gates, tile_amps=16384, min_run=128)
    assert info["fused_passes"] >= 4
    b = q.State(dims, "c64", init=None).set_amplitudes(psi0)
    b.run(gates)
    assert np.array_equal(a.amplitudes(), b.amplitudes())


def block_shape_gates(rng, dims, T, count, max_m):
    # uncontrolled gates on the qudits T (a register block's joint class):
    # dense on one or two of them (classes up to max_m), phases with some
    # factors exactly 1, and cyclic shifts by every amount
    out = []
    while len(out) < count:
        r = rng.random()
        if r < 0.4 or len(T) == 1:
            q = int(rng.choice(T))
            d = dims[q]
            kind = int(rng.integers(4))
            if kind == 0 and d <= max_m:
                out.append(Gate((q,), haar(d, rng)))
            elif kind == 1:
                out.append(Gate((q,), shift(d, int(rng.integers(1, d)))))
            elif kind == 2:
                out.append(Gate((q,), np.diag(np.where(rng.random(d) < 0.3, 1.0, np.exp(2j * np.pi * rng.random(d))))))
            else:
                out.append(Gate((q,), clock(d)))
        else:
            a, b = (int(x) for x in rng.choice(T, 2, replace=False))
            if dims[a] * dims[b] <= max_m:
                out.append(Gate((a, b), haar(dims[a] * dims[b], rng)))
    return out


# Every register-block shape (joint-class dims in ascending order), each on
# qudits spread over a register with other dims around them.
BLOCK_SHAPES = [(2,), (3,), (4,), (5,), (6,), (7,), (2, 2), (2, 3), (2, 4), (2, 5), (2, 6), (2, 7), (3, 3), (3, 4),
                (3, 5), (4, 4), (2, 2, 2), (2, 2, 3), (2, 2, 4)]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_register_blocks_every_shape_bitwise(precision):
    # Register blocks apply runs of uncontrolled gates in registers: the fused
    # result equals one sweep per gate bit for bit (in the given order, and with
    # look-ahead in the planned order) and the oracle within the tolerances.
    q = qd()
    max_m = 4 if precision == "c128" else 7
    rng = np.random.default_rng(2024)
    for shape in BLOCK_SHAPES:
        # the block's qudits at positions 1, 3 (and 5) among qubits and a qutrit
        dims = [2, shape[0], 3, shape[1] if len(shape) > 1 else 2, 2, shape[2] if len(shape) > 2 else 3, 2]
        T = [1, 3, 5][:len(shape)]
        gates = block_shape_gates(rng, dims, T, 24, max_m)
        # a controlled gate in the middle ends one block and starts another
        gates.insert(12, Gate((T[0],), shift(dims[T[0]]), (6,), (1,)))
        psi0 = rand_state(rng, math.prod(dims))
        for reorder in (0, 32):
            passes, order = q.circuit_plan(dims, gates, precision, tile_amps=1024, min_run=2, reorder=reorder,
                                           with_order=True)
            a = q.State(dims, precision, init=None).set_amplitudes(psi0)
            a.run_circuit(gates, tile_amps=1024, min_run=2, reorder=reorder)
            c = q.State(dims, precision, init=None).set_amplitudes(psi0)
            c.run([gates[i] for i in order])
            assert np.array_equal(a.amplitudes(), c.amplitudes()), f"shape {shape}, reorder {reorder}"
            ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                           1j * psi0.imag.astype(np.float32).astype(np.float64))
            for g in gates:
                oracle.apply_gate(dims, ref, g)
            assert_close(a.amplitudes(), ref, precision, f"blocks {shape} reorder {reorder}")
            a.close()
            c.close()




def outer_control_block_gates(rng, dims, T, C, count, max_m):
    # 1-qudit gates on the block qudits T, uncontrolled or with one or two
    # controls on the qudits C (outside small tiles): dense, shifts, phases
    out = []
    while len(out) < count:
        q = int(rng.choice(T))
        d = dims[q]
        kind = int(rng.integers(4))
        if kind == 0 and d <= max_m:
            U = haar(d, rng)
        elif kind == 1:
            U = shift(d, int(rng.integers(1, d)))
        elif kind == 2:
            U = np.diag(np.where(rng.random(d) < 0.3, 1.0, np.exp(2j * np.pi * rng.random(d))))
        else:
            U = clock(d)
        nc = int(rng.integers(3))
        cs = tuple(int(c) for c in rng.choice(C, nc, replace=False))
        out.append(Gate((q,), U, cs, tuple(int(rng.integers(dims[c])) for c in cs)))
    return out


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_register_blocks_with_outer_controls_bitwise(precision):
    # Gates whose controls all lie outside the tile join register blocks; each
    # tile applies only the gates whose outer controls hold on it. Fused equals
    # one sweep per gate bit for bit (given order and planned order) and the
    # oracle within the tolerances.
    q = qd()
    dims = [2] * 5 + [2, 3, 2] + [3, 2, 3, 2]
    T, C = [5, 6, 7], [8, 9, 10, 11]
    max_m = 4 if precision == "c128" else 7
    rng = np.random.default_rng(515)
    gates = outer_control_block_gates(rng, dims, T, C, 60, max_m)
    gates.insert(30, Gate((5, 7), haar(4, rng)))          # an uncontrolled two-qudit gate in the block's qudits
    gates.insert(45, Gate((0,), shift(2), (9,), (1,)))    # a gate outside the block's qudits
    psi0 = rand_state(rng, math.prod(dims))
    for reorder in (0, 64):
        passes, order = q.circuit_plan(dims, gates, precision, tile_amps=256, min_run=32, reorder=reorder,
                                       with_order=True)
        a = q.State(dims, precision, init=None).set_amplitudes(psi0)
        a.run_circuit(gates, tile_amps=256, min_run=32, reorder=reorder)
        c = q.State(dims, precision, init=None).set_amplitudes(psi0)
        c.run([gates[i] for i in order])
        assert np.array_equal(a.amplitudes(), c.amplitudes()), f"reorder {reorder}"
        ref = psi0.copy() if precision == "c128" else (psi0.real.astype(np.float32).astype(np.float64) +
                                                       1j * psi0.imag.astype(np.float32).astype(np.float64))
        for g in gates:
            oracle.apply_gate(dims, ref, g)
        assert_close(a.amplitudes(), ref, precision, f"outer-controlled blocks, reorder {reorder}")
        a.close()
        c.close()
