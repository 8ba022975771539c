"""Sparse block simulation (the paper's sparse variant, Sec. 3): the sparse
oracle is pinned to the dense oracle and to the GHZ closed form at the
register sizes the paper quotes; the GPU form (qd_sparse_*) must reproduce the
sparse oracle's entries exactly (same products without FMA, same summation
order; absent members contribute only signed zeros)."""
import math

import numpy as np
import pytest

import oracle
from oracle import sparse as soracle
from qd_inputs import Gate, circuits, dft, haar, shift


def dense_of(dims, st):
    v = np.zeros(math.prod(dims), dtype=np.complex128)
    for j, a in st.items():
        v[j] = a
    return v


def rand_circuit(rng, dims, count):
    n, out = len(dims), []
    while len(out) < count:
        r = rng.random()
        if r < 0.5:
            t = int(rng.integers(n))
            out.append(Gate((t,), [haar(dims[t], rng), dft(dims[t]), shift(dims[t])][int(rng.integers(3))]))
        elif r < 0.85:
            c, t = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(Gate((t,), shift(dims[t], int(rng.integers(1, dims[t]))), (c,), (int(rng.integers(dims[c])),)))
        else:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            if dims[a] * dims[b] <= 16:
                out.append(Gate((a, b), haar(dims[a] * dims[b], rng)))
    return out


def ghz_gates(d, n):
    """DFT on q0, then X_{+v} on every other qudit controlled on q0 = v."""
    gates = [Gate((0,), dft(d))]
    for q in range(1, n):
        for v in range(1, d):
            gates.append(Gate((q,), shift(d, v), (0,), (v,)))
    return gates


def ghz_closed_form(d, n):
    step = sum(d ** q for q in range(n))
    col = dft(d)[:, 0]
    return {v * step: complex(col[v]) for v in range(d)}


def test_sparse_oracle_equals_dense_oracle():
    rng = np.random.default_rng(1)
    for _ in range(25):
        dims = [int(x) for x in rng.integers(2, 6, size=int(rng.integers(2, 6)))]
        if math.prod(dims) > 3000:
            continue
        gates = rand_circuit(rng, dims, 30)
        assert np.array_equal(dense_of(dims, soracle.run(dims, gates)), oracle.run(dims, gates))


@pytest.mark.parametrize("d,n", [(2, 62), (3, 39), (4, 31), (5, 27), (3, 5)])
def test_sparse_oracle_ghz_closed_form(d, n):
    st = soracle.run([d] * n, ghz_gates(d, n))
    assert st == ghz_closed_form(d, n)


# Registers past the signed 64-bit index of the paper's sparse runs (Sec. 3),
# reached with wider keys (Sec. 4): two key words, and three for 7^45.
WIDE_GHZ = [(2, 100), (3, 63), (4, 50), (5, 43), (7, 45), (2, 126)]


@pytest.mark.parametrize("d,n", WIDE_GHZ)
def test_sparse_oracle_ghz_closed_form_wide(d, n):
    assert d ** n < 2**127
    st = soracle.run([d] * n, ghz_gates(d, n))
    assert st == ghz_closed_form(d, n)


def test_sparse_register_limits_host():
    # D = prod dims as a 128-bit value, and the key words (qudits packed from q0
    # while the product of a word's dims stays below 2^64).
    for dims, words in (([2] * 63, 1), ([2] * 64, 2), ([2] * 126, 2), ([3] * 80, 2), ([4] * 63, 3), ([5] * 54, 2),
                        ([7] * 45, 3), ([7] * 22 + [2] * 3, 2), ([2] * 62, 1)):
        D, w = qd().sparse_dim(dims)
        assert D == math.prod(dims) and w == words, (dims, D, w)
    for dims in ([2] * 125 + [5], [3] * 81, [5] * 55, [7] * 46, [4] * 64):
        with pytest.raises(qd().QDError) as e:
            qd().sparse_dim(dims)
        assert e.value.code == -2  # QD_ERR_DIM_OVERFLOW: D >= 2^127
    for dims in ([], [2] * 127 + [1], [2, 8], [1, 2]):
        with pytest.raises(qd().QDError):
            qd().sparse_dim(dims)


def test_sparse_oracle_drops_exact_zeros():
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)  # real entries: h*h - h*h is exactly 0
    st = soracle.apply([2, 2], soracle.zero_state([2, 2]), (0,), h)
    assert len(st) == 2
    st = soracle.apply([2, 2], st, (0,), h)  # the |1> term cancels exactly and is dropped
    assert set(st) == {0}


# --- GPU ----------------------------------------------------------------------


def qd():
    import paper_2410_17876_amd as q
    return q


def gpu_dict(st):
    keys, amps = st.entries()
    return {int(k): complex(a) for k, a in zip(keys, amps)}



@pytest.mark.gpu
def test_sparse_gpu_equals_sparse_oracle():
    rng = np.random.default_rng(2)
    for i in range(20):
        dims = [int(x) for x in rng.integers(2, 8, size=int(rng.integers(3, 9)))]
        gates = rand_circuit(rng, dims, 40)
        st = qd().SparseState(dims)
        ref = soracle.zero_state(dims)
        for g in gates:
            st.apply_gate(g)
            ref = soracle.apply(dims, ref, g.targets, g.U, g.controls, g.values)
        assert gpu_dict(st) == ref, f"case {i} dims {dims}"
        keys, _ = st.entries()
        assert np.all(np.diff(keys.astype(np.int64)) > 0)
        st.close()


@pytest.mark.gpu
@pytest.mark.parametrize("d,n", [(2, 62), (3, 39), (4, 31), (5, 27)])
def test_sparse_gpu_ghz_at_the_largest_registers(d, n):
    st = qd().SparseState([d] * n)
    for g in ghz_gates(d, n):
        st.apply_gate(g)
    assert st.nnz() == d
    assert gpu_dict(st) == ghz_closed_form(d, n)
    # and back: the inverse circuit returns |0...0> up to the rounding of the
    # DFT's roots of unity, entry for entry as the sparse oracle computes it
    back = list(reversed([g.inverse() for g in ghz_gates(d, n)]))
    for g in back:
        st.apply_gate(g)
    ref = soracle.run([d] * n, back, ghz_closed_form(d, n))
    assert gpu_dict(st) == ref
    assert abs(ref[0] - 1.0) < 1e-15 and all(abs(a) < 1e-15 for j, a in ref.items() if j)
    st.close()


@pytest.mark.gpu
@pytest.mark.parametrize("d,n", WIDE_GHZ)
def test_sparse_gpu_ghz_wide_keys(d, n):
    # GHZ_d beyond 2^64 basis states: multi-word keys, entry for entry against
    # the sparse oracle (Python integers) and the closed form, then back.
    st = qd().SparseState([d] * n)
    assert st.words == (3 if d == 7 else 2)
    gates = ghz_gates(d, n)
    for g in gates:
        st.apply_gate(g)
    assert st.nnz() == d
    assert gpu_dict(st) == ghz_closed_form(d, n) == soracle.run([d] * n, gates)
    back = list(reversed([g.inverse() for g in gates]))
    for g in back:
        st.apply_gate(g)
    assert gpu_dict(st) == soracle.run([d] * n, back, ghz_closed_form(d, n))
    st.close()


WIDE_REGISTERS = [
    [7] * 20 + [2, 3, 5, 7] * 3 + [3] * 10,   # D ~ 2^95: two key words, the first ends inside the 2,3,5,7 run
    [7] * 45,                                 # D ~ 2^126: three key words
    [2, 3] * 30 + [5] * 8,                    # D ~ 2^96: two key words
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(len(WIDE_REGISTERS)))
def test_sparse_gpu_wide_random_circuits(case):
    # Random gates with targets and controls in every key word, gate by gate
    # against the sparse oracle. Superpositions act on five qudits spread over
    # the words (so the state stays within tens of thousands of entries and the
    # oracle stays quick), permutations and controlled shifts anywhere: the state
    # goes from a few entries (one-workgroup form) to thousands (multi-kernel form).
    dims = WIDE_REGISTERS[case]
    n = len(dims)
    S = [0, n // 3, n // 2, 2 * n // 3, n - 1]
    rng = np.random.default_rng(40 + case)
    st = qd().SparseState(dims)
    ref = soracle.zero_state(dims)
    biggest = 1
    for i in range(70):
        r = rng.random()
        if r < 0.35:
            t = int(rng.choice(S))
            g = Gate((t,), haar(dims[t], rng) if rng.random() < 0.7 else dft(dims[t]))
        elif r < 0.85:
            c, t = (int(x) for x in rng.choice(n, 2, replace=False))
            g = Gate((t,), shift(dims[t], int(rng.integers(1, dims[t]))), (c,), (int(rng.integers(dims[c])),))
        else:
            a, b = (int(x) for x in rng.choice(S, 2, replace=False))
            if dims[a] * dims[b] > 16:
                continue
            g = Gate((a, b), haar(dims[a] * dims[b], rng))
        st.apply_gate(g)
        ref = soracle.apply(dims, ref, g.targets, g.U, g.controls, g.values)
        biggest = max(biggest, len(ref) * g.M)
        if i % 10 == 9 or i == 69:
            got = gpu_dict(st)
            print(f"[sparse wide {case}] gate {i}: {len(got)} entries", flush=True)
            assert got == ref, f"gate {i}: {len(got)} vs {len(ref)} entries"
            keys, _ = st.entries()
            assert all(a < b for a, b in zip(keys, keys[1:]))
    if case < 2:
        assert biggest > 1024  # the multi-kernel form ran
    st.close()


@pytest.mark.gpu
def test_sparse_gpu_switches_forms_on_the_true_count():
    # Permutations keep the count, so the host's bound stays tight; dense gates
    # raise the bound past the one-workgroup limit while the true count may
    # stay low (here each DFT is undone), which makes the host read the count
    # back and go on in the one-workgroup form.
    dims = [3] * 70
    st = qd().SparseState(dims)
    ref = soracle.zero_state(dims)
    gates = []
    for q in range(8):
        gates += [Gate((q,), dft(3)), Gate((q,), dft(3).conj().T), Gate((q + 10,), shift(3), (q,), (0,))]
    for g in gates:
        st.apply_gate(g)
        ref = soracle.apply(dims, ref, g.targets, g.U, g.controls, g.values)
    assert gpu_dict(st) == ref
    st.close()


@pytest.mark.gpu
def test_sparse_gpu_gate_list_in_one_call():
    # qd_sparse_apply_circuit equals gate-by-gate application entry for entry; an
    # invalid gate anywhere in the list leaves the state unchanged
    rng = np.random.default_rng(5)
    dims = [3, 2, 5, 2, 4]  # D = 240: a full state stays small for the oracle, and x 16 passes 1024
    gates = rand_circuit(rng, dims, 60)
    a = qd().SparseState(dims).run(gates)
    b = qd().SparseState(dims)
    for g in gates:
        b.apply_gate(g)
    assert gpu_dict(a) == gpu_dict(b) == soracle.run(dims, gates)
    before = gpu_dict(a)
    with pytest.raises(qd().QDError):
        a.run(gates[:5] + [Gate((0, 0), np.eye(9))] + gates[5:])  # a repeated target
    assert gpu_dict(a) == before
    a.close()
    b.close()


@pytest.mark.gpu
def test_sparse_gpu_errors_leave_state_unchanged(monkeypatch):
    rng = np.random.default_rng(3)
    st = qd().SparseState([5, 5, 3])
    st.apply((0,), dft(5))
    before = gpu_dict(st)
    monkeypatch.setenv("QD_CHECK_UNITARY", "1")  # a non-unitary gate is refused when checking is on
    with pytest.raises(qd().QDError):
        st.apply((1,), 2.0 * dft(5))
    monkeypatch.delenv("QD_CHECK_UNITARY")
    with pytest.raises(qd().QDError):
        st.apply((0, 1), haar(25, rng))  # 25 > 16 amplitudes per class
    with pytest.raises(qd().QDError):
        st.apply((0, 0), haar(25, rng))
    with pytest.raises(qd().QDError):
        st.apply((2,), haar(3, rng), (2,), (1,))
    assert gpu_dict(st) == before
    st.close()


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["ghz2_62", "ghz5_27", "ghz7_45", "random"])
def test_sparse_gpu_runs_equal_gate_by_gate(case):
    # A gate list (qd_sparse_apply_circuit) applies runs of small gates in one
    # launch with the entries kept in LDS; the result must equal gate-by-gate
    # application entry for entry, and the sparse oracle.
    if case == "random":
        rng = np.random.default_rng(77)
        dims = [3, 2, 5, 2, 4, 3]
        gates = rand_circuit(rng, dims, 90)
    else:
        d, n = {"ghz2_62": (2, 62), "ghz5_27": (5, 27), "ghz7_45": (7, 45)}[case]
        dims = [d] * n
        fwd = ghz_gates(d, n)
        gates = fwd + list(reversed([g.inverse() for g in fwd]))
    a = qd().SparseState(dims).run(gates)
    b = qd().SparseState(dims)
    for g in gates:
        b.apply_gate(g)
    assert gpu_dict(a) == gpu_dict(b) == soracle.run(dims, gates)
    a.close()
    b.close()
