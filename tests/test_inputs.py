"""The seeded input generators: determinism and the properties the workloads state."""
import math

import numpy as np

from qd_inputs import circuits, clock, dft, haar, shift, states


def test_gate_matrices_unitary():
    rng = np.random.default_rng(0)
    for d in range(2, 8):
        for U in (dft(d), shift(d), clock(d), haar(d, rng), haar(d * d, rng)):
            np.testing.assert_allclose(U @ U.conj().T, np.eye(U.shape[0]), atol=1e-13)


def test_shift_direction():
    # X_{+1}|j> = |j+1 mod d>: column j holds a 1 in row (j+1) mod d (paper Sec. 2.2).
    X = shift(5, 2)
    for j in range(5):
        assert X[(j + 2) % 5, j] == 1 and np.count_nonzero(X[:, j]) == 1


def test_circuits_deterministic_and_well_formed():
    for make in (circuits.plain, circuits.large, circuits.fused):
        dims, g1 = make()
        _, g2 = make()
        assert len(g1) == len(g2)
        for a, b in zip(g1, g2):
            assert a.targets == b.targets and a.controls == b.controls and a.values == b.values
            assert np.array_equal(a.U, b.U)
            assert a.M == math.prod(dims[t] for t in a.targets)
            assert len(set(a.targets + a.controls)) == len(a.targets) + len(a.controls)
            assert all(0 <= v < dims[c] for c, v in zip(a.controls, a.values))
    dims, gates = circuits.large()
    assert math.prod(dims) == 2**14 * 3**8 * 4**2 and len(gates) == 500
    kinds = [g.kind for g in gates]
    assert 20 < kinds.count("haar2") < 80
    dims, gates = circuits.fused()
    assert dims == [5] * 12 and {g.M for g in gates} == {25, 125}


def test_batched_and_served_specs():
    specs = circuits.batched_specs()
    assert len(specs) == 512
    assert all(6 <= len(s.dims) <= 16 and s.D <= 10**6 and 100 <= s.depth <= 1000 for s in specs)
    assert all(set(s.dims) <= {2, 3, 4, 5} for s in specs)
    reqs = circuits.served_requests(qps=10.0, count=200)
    assert all(1e3 <= r.spec.D <= 1e8 for r in reqs)
    assert all(b.arrival >= a.arrival for a, b in zip(reqs, reqs[1:]))


def test_gaussian_state_indexable_and_normalised():
    G = states.GaussianState(3 * 2**20 + 12345, seed=5, chunk=2**20)
    full = G.full()
    assert abs(math.fsum((np.abs(full) ** 2).tolist()) - 1.0) < 1e-12
    idx = np.array([0, 1, 2**20 - 1, 2**20, 3 * 2**20 + 12344, 777777])
    assert np.array_equal(G.values(idx), full[idx])
    G2 = states.GaussianState(3 * 2**20 + 12345, seed=5, chunk=2**20)
    assert np.array_equal(G2.values(idx), full[idx])


def test_labelled_state_exact_in_fp32():
    v = states.labelled(2**40 - 5, 10)
    assert np.array_equal(v.real.astype(np.float32).astype(np.float64), v.real)
    assert np.array_equal(v.imag.astype(np.float32).astype(np.float64), v.imag)
