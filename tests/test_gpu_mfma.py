"""Matrix-core path (dense gates with 17 <= M <= 128: complex64 on FP32 MFMA,
complex128 on FP64 MFMA, its 256 x 256 real form streamed from L2 above 64
members) against the FP64 oracle, and the ququint workload: 2- and 3-qudit
Haar gates (25x25, 125x125).

Tolerance: complex64, max-abs <= 2e-5 and <= 1e-5 of the largest amplitude,
per gate layer (a layer = one gate, as each gate is one launch here);
complex128, max-abs <= 1e-12."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, gpu_values, rand_state, upload_chunks
from qd_inputs import Gate, circuits, haar, states

pytestmark = pytest.mark.gpu


def qd():
    import paper_2410_17876_amd as q
    return q


def round32(v):
    return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)


CASES = [  # (dims, targets): M = 18, 25, 27, 36, 48, 49, 64, 100, 125, 126, 25, 25, 25, 125
    ([2, 3, 3, 2, 5, 2, 3], [1, 2, 0]),
    ([5, 2, 5, 3, 2, 2, 3], [0, 2]),
    ([3, 3, 2, 3, 5, 2, 2], [0, 1, 3]),
    ([6, 2, 6, 3, 2, 5], [2, 0]),
    ([4, 3, 2, 4, 5, 2], [3, 1, 0]),
    ([7, 3, 7, 2, 2, 3], [2, 0]),
    ([4, 4, 4, 3, 2, 5], [0, 1, 2]),
    ([5, 3, 5, 4, 2, 3], [2, 3, 0]),
    ([5, 5, 5, 3, 2, 2, 2], [0, 1, 2]),
    ([2, 7, 6, 3, 3, 2], [1, 2, 3]),
    # free qudits below the lowest target (gather order with a free low run F)
    ([3, 5, 5, 2, 2, 3, 2], [1, 2]),       # F = 3
    ([2, 2, 5, 5, 3, 2, 2], [3, 2]),       # F = 4
    ([5, 5, 5, 5, 2, 3], [2, 3]),          # F = 25: 125 classes per tile
    ([2, 5, 5, 5, 3, 2], [1, 2, 3]),       # F = 2, M = 125
]


def _m(dims, targets):
    return math.prod(dims[t] for t in targets)


PCASES = [(d, t, "c64") for d, t in CASES] + [(d, t, "c128") for d, t in CASES]


@pytest.mark.parametrize("dims,targets,precision", PCASES)
def test_mfma_gate_vs_oracle(dims, targets, precision):
    rng = np.random.default_rng(sum(dims) * 7 + len(targets))
    D = math.prod(dims)
    M = _m(dims, targets)
    assert qd().gate_info(dims, targets, haar(M, rng), precision=precision)["kernel"] == "block_mfma"
    psi0 = rand_state(rng, D)
    U = haar(M, rng)
    rest = [q for q in range(len(dims)) if q not in targets]
    start = round32(psi0) if precision == "c64" else psi0
    for controls, values in (((), ()), ((rest[-1],), (dims[rest[-1]] - 1,))):
        st = qd().State(dims, precision, init=None).set_amplitudes(psi0)
        st.apply(targets, U, controls, values)
        ref = oracle.apply(dims, start.copy(), targets, U, controls, values)  # in place: on a copy
        assert_close(st.amplitudes(), ref, precision, f"M={M} controls={controls}")


def test_mfma_c128_roundtrip_and_determinism():
    # FP64 matrix cores: 64x64 (three ququarts), 25x25 (two ququints) and, streamed,
    # 75x75 and 100x100 blocks,
    # with ragged last tiles (D / M classes is no multiple of the tile width)
    rng = np.random.default_rng(9)
    dims = [4, 5, 4, 5, 4, 3, 2]
    psi0 = rand_state(rng, math.prod(dims))
    gates = [Gate((4, 0, 2), haar(64, rng)), Gate((1, 3), haar(25, rng)), Gate((3, 1), haar(25, rng)),
             Gate((2, 4, 0), haar(64, rng)), Gate((0, 2, 4), haar(64, rng), (5,), (2,)),
             Gate((1, 3, 5), haar(75, rng)), Gate((3, 2, 1), haar(100, rng), (6,), (1,))]
    for g in gates:
        assert qd().gate_info(dims, g.targets, g.U, precision="c128")["kernel"] == "block_mfma"
    a = qd().State(dims, "c128", init=None).set_amplitudes(psi0).run(gates)
    b = qd().State(dims, "c128", init=None).set_amplitudes(psi0).run(gates)
    assert np.array_equal(a.amplitudes(), b.amplitudes())
    assert_close(a.amplitudes(), oracle.run(dims, gates, psi0.copy()), "c128", "5 gates")
    for g in reversed(gates):
        a.apply_gate(g.inverse())
    assert_close(a.amplitudes(), psi0, "c128", "roundtrip")


def test_mfma_roundtrip_and_determinism():
    rng = np.random.default_rng(3)
    dims = [5, 5, 5, 5, 3, 2]
    psi0 = rand_state(rng, math.prod(dims))
    gates = [Gate(tuple(int(x) for x in rng.choice(4, 3, replace=False)), haar(125, rng)) for _ in range(6)]
    gates += [Gate(tuple(int(x) for x in rng.choice(4, 2, replace=False)), haar(25, rng)) for _ in range(6)]
    a = qd().State(dims, "c64", init=None).set_amplitudes(psi0).run(gates)
    b = qd().State(dims, "c64", init=None).set_amplitudes(psi0).run(gates)
    assert np.array_equal(a.amplitudes(), b.amplitudes())
    for g in reversed(gates):
        a.apply_gate(g.inverse())
    assert_close(a.amplitudes(), round32(psi0), "c64", "roundtrip")


def test_ququint_circuit_per_layer_vs_oracle():
    # The ququint workload's gate mix on 8 ququints (D = 390625), GPU and oracle
    # advanced in lockstep from |0..0>; the error is recorded after every layer.
    dims, gates = circuits.fused(dims=[5] * 8, n_gates=60)
    st = qd().State(dims, "c64")
    ref = oracle.zero_state(dims)
    errs = []
    for g in gates:
        st.apply_gate(g)
        oracle.apply_gate(dims, ref, g)
        got = st.amplitudes()
        errs.append(float(np.max(np.abs(got - ref))))
        assert_close(got, ref, "c64", f"layer {len(errs) - 1} ({g.kind} on {g.targets})")
    print(f"[ququint 5^8] per-layer max-abs error: first {errs[0]:.2e}, last {errs[-1]:.2e}, max {max(errs):.2e}")


def test_64bit_path_mfma():
    # D >= 2^31 (5^14 = 6.1e9 would be 49 GB in c64; 5^13 x 2 = 2.4e9 suffices).
    import torch

    dims = [5] * 13 + [2]
    D = math.prod(dims)
    assert D >= 2**31
    st = qd().State(dims, "c64", init=None)
    upload_chunks(st, lambda s, c: states.labelled(s, c), chunk=1 << 24)
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.integers(0, D, size=3000), [0, D - 1]])
    for targets in ((12, 3, 7), (0, 13)):
        M = math.prod(dims[t] for t in targets)
        g = Gate(targets, haar(M, rng))
        st.apply_gate(g)
        want = oracle.apply_sampled(dims, g, idx, states.labelled_at)
        got = gpu_values(st, idx)
        assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want)), targets
        st.apply_gate(g.inverse())
    st.close()
    del st
    torch.cuda.empty_cache()


def test_64bit_path_mfma_c128():
    # D = 5^13 x 2 >= 2^31 in complex128 (39 GB): 64-bit class bases and offsets
    import torch

    dims = [5] * 13 + [2]
    D = math.prod(dims)
    st = qd().State(dims, "c128", init=None)
    upload_chunks(st, lambda s, c: states.labelled(s, c), chunk=1 << 24)
    rng = np.random.default_rng(12)
    idx = np.concatenate([rng.integers(0, D, size=3000), [0, D - 1]])
    for targets in ((12, 3), (0, 13, 6), (12, 3, 7)):
        M = math.prod(dims[t] for t in targets)
        g = Gate(targets, haar(M, rng))
        assert qd().gate_info(dims, targets, g.U, precision="c128")["kernel"] == "block_mfma"
        st.apply_gate(g)
        want = oracle.apply_sampled(dims, g, idx, states.labelled_at)
        # labelled amplitudes reach 2^20: bound the error relative to the largest
        err = float(np.max(np.abs(gpu_values(st, idx) - want)))
        assert err <= 1e-13 * float(np.max(np.abs(want))), (targets, err)
        st.apply_gate(g.inverse())
    st.close()
    del st
    torch.cuda.empty_cache()


def test_full_ququint_register_sampled():
    # The full workload register: 12 ququints (D = 2.44e8). Single gates of the
    # workload on a seeded Gaussian input, sampled outputs vs the oracle's sampled
    # form (inputs straight from the generator), then the 300-gate circuit and its
    # inverse return the input.
    import torch

    dims, gates = circuits.fused()
    D = math.prod(dims)
    G = states.GaussianState(D, seed=77)
    G.cache_chunks = 240
    st = qd().State(dims, "c64", init=None)
    G.fill(lambda start, vals: st.set_interleaved(vals, start))
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.integers(0, D, size=2000), [0, D - 1]])
    inp = lambda ix: round32(G.values(ix))
    for g in gates[:8]:
        st.apply_gate(g)
        assert_close(gpu_values(st, idx), oracle.apply_sampled(dims, g, idx, inp), "c64", f"{g.kind} {g.targets}")
        st.apply_gate(g.inverse())
    st.run(gates)
    assert abs(st.norm() - 1.0) < 1e-4
    for g in reversed(gates):
        st.apply_gate(g.inverse())
    got = gpu_values(st, idx)
    err = float(np.max(np.abs(got - inp(idx))))
    print(f"[ququint 5^12] 600-gate roundtrip max-abs error {err:.3e}")
    assert_close(got, inp(idx), "c64", "600-gate ququint roundtrip")
    st.close()
    del st
    torch.cuda.empty_cache()


def test_mfma_control_below_targets():
    # a control on q0 under low targets: the plain class order (no free low run)
    rng = np.random.default_rng(41)
    dims = [3, 5, 5, 2, 2, 3, 2]
    psi0 = rand_state(rng, math.prod(dims))
    U = haar(25, rng)
    st = qd().State(dims, "c64", init=None).set_amplitudes(psi0)
    st.apply([1, 2], U, [0], [2])
    assert_close(st.amplitudes(), oracle.apply(dims, round32(psi0), [1, 2], U, [0], [2]), "c64", "control on q0")
