"""qd_norm_noalloc, the norm for callers that cannot allocate: through the C
ABI, its values must equal qd_norm's bit for bit (the same fixed-order FP64
reduction), on two calls in a row, the second with a smaller input (fewer and
smaller states), so that the second call runs on the partial sums the first
left in the library's fixed scratch array."""
import ctypes as C
import math

import numpy as np
import pytest

from gpu_util import rand_state

pytestmark = pytest.mark.gpu


def qd():
    import paper_2410_17876_amd as q
    return q


def abi_norms(states, out):
    lib = qd().lib
    hs = (C.c_void_p * len(states))(*[st.handle for st in states])
    rc = lib.qd_norm_noalloc(hs, len(states), C.c_void_p(out.data_ptr()))
    assert rc == 0, lib.qd_last_error().decode()


def test_norm_noalloc_equals_norm_on_two_calls():
    import torch

    rng = np.random.default_rng(91)
    shapes = [([2] * 20 + [3] * 2, "c128"), ([5] * 8, "c64"), ([3, 4, 7, 2, 2, 5], "c128"), ([2] * 24, "c64"),
              ([7] * 7, "c128")]
    states = []
    for dims, p in shapes:
        st = qd().State(dims, p, init=None)
        D = math.prod(dims)
        chunk = 1 << 22
        for s0 in range(0, D, chunk):  # an unnormalised Gaussian state, so the norms differ
            c = min(chunk, D - s0)
            st.set_amplitudes(rand_state(rng, c) * (1.0 + rng.random()), s0)
        states.append(st)
    out = torch.full((len(states),), float("nan"), dtype=torch.float64, device="cuda")
    abi_norms(states, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array([st.norm() for st in states])
    print(f"[noalloc] first call, {len(states)} states: {got}", flush=True)
    assert np.array_equal(got, want), (got, want)
    # second call: fewer, smaller states (the scratch keeps the first call's partials)
    small = [qd().State([3, 2, 2], "c128", init=None).set_amplitudes(rand_state(rng, 12) * 3.0),
             qd().State([2, 5], "c64", init=None).set_amplitudes(rand_state(rng, 10) * 0.5)]
    out2 = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    abi_norms(small, out2)
    torch.cuda.synchronize()
    got2 = out2.cpu().numpy()
    want2 = np.array([st.norm() for st in small])
    print(f"[noalloc] second call, 2 small states: {got2}", flush=True)
    assert np.array_equal(got2, want2), (got2, want2)
    for st in states + small:
        st.close()


def test_norm_noalloc_rejects_bad_arguments():
    import torch

    st = qd().State([2, 3], "c128")
    out = torch.zeros(65, dtype=torch.float64, device="cuda")
    lib = qd().lib
    many = (C.c_void_p * 65)(*([st.handle] * 65))
    assert lib.qd_norm_noalloc(many, 65, C.c_void_p(out.data_ptr())) == -5  # more than 64 states
    assert b"at most" in lib.qd_last_error()
    two = (C.c_void_p * 2)(st.handle, st.handle)
    assert lib.qd_norm_noalloc(two, 2, C.c_void_p(out.data_ptr())) == -1  # listed twice
    assert lib.qd_norm_noalloc(two, 0, C.c_void_p(out.data_ptr())) == -1
    assert lib.qd_norm_noalloc(two, 1, None) == -1
    st.close()
