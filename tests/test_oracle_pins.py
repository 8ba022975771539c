"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked example (golden file), a tensor-contraction and a Kronecker-product
formulation (numpy library routines), closed forms, and invariants. The
mutation tests at the end plant plausible mistakes in a copy of the oracle's
source and confirm that these pins catch them.
"""
import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from brute import kron_operator, tensor_apply
from qd_inputs import Gate, circuits, clock, dagger, dft, haar, shift, states

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_state(rng, D):
    v = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return v / np.linalg.norm(v)


def rand_gate(rng, dims, k_max=3, m_max=2, adjacent=False):
    n = len(dims)
    k = int(rng.integers(1, min(k_max, n) + 1))
    if adjacent:
        t0 = int(rng.integers(0, n - k + 1))
        targets = list(range(t0, t0 + k))
    else:
        targets = [int(x) for x in rng.choice(n, k, replace=False)]
    rest = [q for q in range(n) if q not in targets]
    m = int(rng.integers(0, min(m_max, len(rest)) + 1))
    controls = [int(x) for x in rng.choice(rest, m, replace=False)] if m else []
    values = [int(rng.integers(dims[c])) for c in controls]
    M = int(np.prod([dims[t] for t in targets]))
    return Gate(tuple(targets), haar(M, rng), tuple(controls), tuple(values))


def rand_dims(rng, n_max=5, D_max=2000):
    while True:
        n = int(rng.integers(1, n_max + 1))
        dims = [int(x) for x in rng.integers(2, 8, size=n)]
        if math.prod(dims) <= D_max:
            return dims


@pytest.fixture(autouse=True, params=[1, 4], ids=["1thread", "4threads"])
def oracle_threads(request):
    """Every pin runs with the oracle's scan on one thread and on four."""
    with oracle.threads(request.param):
        yield request.param


def test_thread_split_is_bitwise():
    # The scan over base indices may run on several threads: classes are
    # disjoint (Sec. 2.3), so every amplitude gets the same operations in the
    # same order and the result must not change by a single bit.
    rng = np.random.default_rng(77)
    dims = [2, 3, 5, 2, 4, 7, 3, 2, 2, 3]
    psi0 = rand_state(rng, math.prod(dims))
    gates = [rand_gate(rng, dims, m_max=3) for _ in range(40)]
    masked = [(g.targets, g.U, g.controls, [(1 << dims[c]) - 1 - (1 << v) for c, v in zip(g.controls, g.values)])
              for g in gates[:10]]
    out = []
    for n in (1, 2, 7):
        with oracle.threads(n):
            psi = oracle.run(dims, gates, psi0)
            for t, U, c, mk in masked:
                oracle.apply_masked(dims, psi, t, U, c, mk)
            out.append(psi)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


# --- worked example (Sec. 2.5) -------------------------------------------------

def load_worked_example():
    rows = []
    with open(os.path.join(GOLDEN, "worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "dims":
                dims = [int(x) for x in parts[1:]]
            elif parts[0].startswith("gate"):
                continue
            else:
                j, x0, x1 = int(parts[0]), int(parts[1]), int(parts[2])
                num, den = parts[3].split("/")
                rows.append((j, x0, x1, int(num) / int(den)))
    return dims, rows


def test_worked_example_golden():
    dims, rows = load_worked_example()
    psi = oracle.zero_state(dims)
    oracle.apply(dims, psi, [1], dft(3))
    oracle.apply(dims, psi, [0], shift(2, 1), [1], [2])
    expected = np.zeros(6, dtype=np.complex128)
    for j, x0, x1, p in rows:
        assert j == x0 + dims[0] * x1
        expected[j] = math.sqrt(p)
    np.testing.assert_allclose(psi, expected, rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.probabilities(psi), np.abs(expected) ** 2, rtol=0, atol=1e-15)


def test_worked_example_grouping():
    # Fig. 2: grouping by q1 gives blocks {i00,i01},{i10,i11},{i20,i21} of size d0 = 2
    # (block size = product of less significant dims, Sec. 2.3); a class takes the
    # element at the same offset in each block (Table 2): {0,2,4} and {1,3,5}.
    members, row = oracle.class_members([2, 3], [1], [], [], np.arange(6))
    classes = {tuple(sorted(m)) for m in members.tolist()}
    assert classes == {(0, 2, 4), (1, 3, 5)}
    assert row.tolist() == [0, 0, 1, 1, 2, 2]


# --- brute-force formulations ---------------------------------------------------

def test_oracle_matches_tensor_contraction():
    rng = np.random.default_rng(7)
    for _ in range(300):
        dims = rand_dims(rng)
        g = rand_gate(rng, dims)
        psi0 = rand_state(rng, math.prod(dims))
        got = oracle.apply(dims, psi0.copy(), g.targets, g.U, g.controls, g.values)
        want = tensor_apply(dims, psi0, g.targets, g.U, g.controls, g.values)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_oracle_matches_kron_operator():
    rng = np.random.default_rng(8)
    for _ in range(150):
        dims = rand_dims(rng, n_max=4, D_max=400)
        g = rand_gate(rng, dims, adjacent=True)
        psi0 = rand_state(rng, math.prod(dims))
        G = kron_operator(dims, g.targets, g.U, g.controls, g.values)
        got = oracle.apply(dims, psi0.copy(), g.targets, g.U, g.controls, g.values)
        np.testing.assert_allclose(got, G @ psi0, rtol=0, atol=1e-13)


def test_target_order_convention():
    # kron(A, B) on targets [t0, t1] = B on t0, then A on t1 (first target least significant).
    rng = np.random.default_rng(9)
    dims = [3, 2, 4, 3]
    A, B = haar(dims[2], rng), haar(dims[1], rng)
    psi0 = rand_state(rng, math.prod(dims))
    got = oracle.apply(dims, psi0.copy(), [1, 2], np.kron(A, B))
    ref = oracle.apply(dims, psi0.copy(), [1], B)
    ref = oracle.apply(dims, ref, [2], A)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    # Listing the targets the other way round swaps the roles of the factors.
    got2 = oracle.apply(dims, psi0.copy(), [2, 1], np.kron(B, A))
    np.testing.assert_allclose(got2, ref, rtol=0, atol=1e-14)


def test_whole_plain_circuit_gate_by_gate():
    dims, gates = circuits.plain()
    psi = oracle.zero_state(dims)
    ref = psi.copy()
    for g in gates:
        oracle.apply_gate(dims, psi, g)
        ref = tensor_apply(dims, ref, g.targets, g.U, g.controls, g.values)
        np.testing.assert_allclose(psi, ref, rtol=0, atol=1e-12)


# --- closed forms and invariants ------------------------------------------------

def test_shift_power_is_identity_bit_exact():
    rng = np.random.default_rng(10)
    for dims in ([2, 3, 5], [7, 2], [4, 6, 3]):
        psi0 = rand_state(rng, math.prod(dims))
        for t in range(len(dims)):
            psi = psi0.copy()
            for _ in range(dims[t]):
                oracle.apply(dims, psi, [t], shift(dims[t], 1))
            assert np.array_equal(psi, psi0)


def test_shift_closed_form_index_labelled():
    # X_{+1} on t: psi'[j] = psi[j with digit t replaced by (digit - 1) mod d_t].
    dims = [3, 2, 5, 4, 2]
    D = math.prod(dims)
    s = np.cumprod([1] + dims[:-1])
    psi0 = states.labelled(0, D)
    j = np.arange(D)
    for t in range(len(dims)):
        psi = oracle.apply(dims, psi0.copy(), [t], shift(dims[t], 1))
        dig = (j // s[t]) % dims[t]
        src = j - dig * s[t] + ((dig - 1) % dims[t]) * s[t]
        assert np.array_equal(psi, psi0[src])


def test_dft_fourth_power_and_clock_power():
    rng = np.random.default_rng(11)
    dims = [3, 5, 2, 7]
    psi0 = rand_state(rng, math.prod(dims))
    for t in range(len(dims)):
        psi = psi0.copy()
        for _ in range(4):
            oracle.apply(dims, psi, [t], dft(dims[t]))
        np.testing.assert_allclose(psi, psi0, rtol=0, atol=1e-14)
        psi = psi0.copy()
        for _ in range(dims[t]):
            oracle.apply(dims, psi, [t], clock(dims[t]))
        np.testing.assert_allclose(psi, psi0, rtol=0, atol=1e-14)


def test_dft_everywhere_is_uniform():
    dims = [2, 3, 4, 5, 7]
    D = math.prod(dims)
    psi = oracle.zero_state(dims)
    for t in range(len(dims)):
        oracle.apply(dims, psi, [t], dft(dims[t]))
    np.testing.assert_allclose(psi, np.full(D, 1 / math.sqrt(D)), rtol=0, atol=1e-15)


def test_weyl_commutation():
    # Z X = w X Z on one qudit, w = exp(2 pi i / d).
    rng = np.random.default_rng(12)
    for d in range(2, 8):
        dims = [d, 3]
        psi0 = rand_state(rng, 3 * d)
        a = oracle.apply(dims, oracle.apply(dims, psi0.copy(), [0], shift(d)), [0], clock(d))
        b = oracle.apply(dims, oracle.apply(dims, psi0.copy(), [0], clock(d)), [0], shift(d))
        np.testing.assert_allclose(a, np.exp(2j * np.pi / d) * b, rtol=0, atol=1e-14)


def test_roundtrip_and_norm():
    rng = np.random.default_rng(13)
    for _ in range(50):
        dims = rand_dims(rng)
        gates = [rand_gate(rng, dims) for _ in range(10)]
        psi0 = rand_state(rng, math.prod(dims))
        psi = psi0.copy()
        for g in gates:
            oracle.apply_gate(dims, psi, g)
        assert abs(oracle.norm(psi) - 1.0) < 1e-13
        for g in reversed(gates):
            oracle.apply_gate(dims, psi, g.inverse())
        np.testing.assert_allclose(psi, psi0, rtol=0, atol=1e-13)


def test_non_matching_controls_untouched():
    # Sec. 2.4: the gate only acts where floor(j / b_k) mod d_k = v_k for every control.
    rng = np.random.default_rng(14)
    dims = [3, 4, 2, 5]
    s = np.cumprod([1] + dims[:-1])
    D = math.prod(dims)
    j = np.arange(D)
    psi0 = rand_state(rng, D)
    psi = oracle.apply(dims, psi0.copy(), [2], haar(2, rng), [0, 3], [2, 4])
    hold = ((j // s[0]) % 3 == 2) & ((j // s[3]) % 5 == 4)
    assert np.array_equal(psi[~hold], psi0[~hold])
    assert not np.allclose(psi[hold], psi0[hold])


def test_norm_and_probabilities_against_fsum():
    rng = np.random.default_rng(15)
    psi = rand_state(rng, 999) * 3.7
    p = oracle.probabilities(psi)
    want = [v.real * v.real + v.imag * v.imag for v in psi]
    assert np.array_equal(p, np.array(want))
    assert abs(oracle.norm(psi) - math.sqrt(math.fsum(want))) <= 1e-15 * 3.7


def test_sampled_matches_full():
    rng = np.random.default_rng(16)
    for _ in range(100):
        dims = rand_dims(rng)
        D = math.prod(dims)
        g = rand_gate(rng, dims)
        psi0 = rand_state(rng, D)
        full = oracle.apply(dims, psi0.copy(), g.targets, g.U, g.controls, g.values)
        idx = rng.integers(0, D, size=40)
        got = oracle.apply_sampled(dims, g, idx, lambda ix: psi0[ix])
        assert np.array_equal(got, full[idx])


def test_dimension_limits_of_64bit_index():
    # Sec. 3: the largest registers run were 62 qubits, 39 qutrits, 31 ququads and
    # 27 ququints, limited by a signed 64-bit basis index: exactly the largest n
    # with d^n < 2^63.
    for d, n_max in ((2, 62), (3, 39), (4, 31), (5, 27)):
        assert oracle.dim([d] * n_max) == d ** n_max
        assert oracle.dim([d] * (n_max + 1)) == -1
    assert oracle.dim([1, 2]) == -1 and oracle.dim([8]) == -1


def test_invalid_gates_rejected():
    dims = [2, 3]
    psi = oracle.zero_state(dims)
    with pytest.raises(ValueError):
        oracle.apply(dims, psi, [0, 0], np.eye(4))
    with pytest.raises(ValueError):
        oracle.apply(dims, psi, [0], np.eye(2), [0], [1])
    with pytest.raises(ValueError):
        oracle.apply(dims, psi, [0], np.eye(2), [1], [3])
    with pytest.raises(ValueError):
        oracle.apply(dims, psi, [2], np.eye(2))


# --- mutation tests: plant mistakes in a copy of the oracle ---------------------

MUTANTS = {
    "transposed_U": ("U[2 * (r * M + a)], ui = U[2 * (r * M + a) + 1];\n            double xr = x[2 * a]",
                     "U[2 * (a * M + r)], ui = U[2 * (a * M + r) + 1];\n            double xr = x[2 * a]"),
    "conjugate_sign": ("yi = yi + (ur * xi + ui * xr);\n        }\n        y[2 * r]",
                       "yi = yi + (ur * xi - ui * xr);\n        }\n        y[2 * r]"),
    "dropped_term": ("yr = yr + (ur * xr - ui * xi);\n            yi = yi + (ur * xi + ui * xr);\n        }\n        y[2 * r]",
                     "yr = yr + (ur * xr);\n            yi = yi + (ur * xi + ui * xr);\n        }\n        y[2 * r]"),
    "target_order": ("off += (int64_t)(a % d) * s[targets[l]];",
                     "off += (int64_t)(a % d) * s[targets[k - 1 - l]];"),
    "control_ignored": ("if (!base || !controls_hold(j, m, controls, cvals, dims, s)) continue;",
                        "if (!base) continue;"),
    "block_size_off_by_one": ("for (int i = 1; i < n; ++i) s[i] = s[i - 1] * dims[i - 1];",
                              "for (int i = 1; i < n; ++i) s[i] = s[i - 1] * dims[i];"),
}


def _pins_pass(L) -> bool:
    """Run the tensor-contraction and worked-example pins against library L."""
    import ctypes as C
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
    L.oracle_apply.argtypes = [C.c_int, i32p, f64p, C.c_int, i32p, C.c_int, i32p, i32p, f64p]
    L.oracle_apply.restype = C.c_int

    def ap(dims, psi, g):
        i32 = lambda x: np.asarray(list(x) or [0], dtype=np.int32)
        rc = L.oracle_apply(len(dims), i32(dims), psi.view(np.float64), len(g.targets), i32(g.targets),
                            len(g.controls), i32(g.controls), i32(g.values),
                            np.ascontiguousarray(g.U).view(np.float64).reshape(-1))
        assert rc == 0

    rng = np.random.default_rng(17)
    for _ in range(200):
        dims = rand_dims(rng)
        g = rand_gate(rng, dims)
        psi0 = rand_state(rng, math.prod(dims))
        psi = psi0.copy()
        ap(dims, psi, g)
        if not np.allclose(psi, tensor_apply(dims, psi0, g.targets, g.U, g.controls, g.values),
                           rtol=0, atol=1e-12):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    import ctypes as C
    src = open(os.path.join(os.path.dirname(oracle.__file__), "qd_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib), str(path), "-lm"],
                   check=True)
    assert not _pins_pass(C.CDLL(str(lib)))


def test_unmutated_oracle_passes_mutation_harness():
    import ctypes as C
    assert _pins_pass(C.CDLL(oracle._build.LIB))
