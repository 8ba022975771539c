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
def test_sparse_gpu_errors_leave_state_unchanged():
    rng = np.random.default_rng(3)
    st = qd().SparseState([5, 5, 3])
    st.apply((0,), dft(5))
    before = gpu_dict(st)
    with pytest.raises(qd().QDError):
        st.apply((0, 1), haar(25, rng))  # 25 > 16 amplitudes per class
    with pytest.raises(qd().QDError):
        st.apply((0, 0), haar(25, rng))
    with pytest.raises(qd().QDError):
        st.apply((2,), haar(3, rng), (2,), (1,))
    assert gpu_dict(st) == before
    st.close()
