"""Helpers shared by the GPU tests (test plumbing only)."""
import math

import numpy as np

TOL = {"c128": 1e-12, "c64": 2e-5}


def gpu_values(st, idx) -> np.ndarray:
    """Amplitudes of a library state at the given indices (torch gather)."""
    import torch

    t = torch.as_tensor(np.asarray(idx, dtype=np.int64), device=st.device)
    v = st.buffer.view(-1, 2)[t].double().cpu().numpy()
    return v[:, 0] + 1j * v[:, 1]


def upload_chunks(st, producer, chunk=1 << 22):
    """Upload a state given by producer(start, count) -> complex128 values."""
    for start in range(0, st.D, chunk):
        c = min(chunk, st.D - start)
        st.set_amplitudes(producer(start, c), start)


def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0


def assert_close(got, want, precision, label=""):
    err = max_abs(got, want)
    scale = float(np.max(np.abs(want))) if np.size(want) else 1.0
    tol = TOL[precision]
    assert err <= tol, f"{label}: max-abs error {err:.3e} > {tol:.1e} ({precision})"
    if precision == "c64":
        # The absolute bound is loose for small amplitudes; also bound the error
        # relative to the largest amplitude (FP32 rounding of a few ops per gate).
        assert err <= 1e-5 * scale, f"{label}: relative error {err / scale:.3e} > 1e-5 (c64)"


def rand_state(rng, D):
    v = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return v / np.linalg.norm(v)


def rand_monomial(rng, M, phases=True, fixed=0):
    """Random permutation-with-phases matrix; `fixed` leading identity columns."""
    perm = np.arange(M)
    tail = rng.permutation(M - fixed) + fixed
    perm[fixed:] = tail
    U = np.zeros((M, M), dtype=np.complex128)
    for a in range(M):
        lam = np.exp(2j * np.pi * rng.random()) if (phases and a >= fixed) else 1.0
        U[perm[a], a] = lam
    return U


def prod(x):
    return int(math.prod(x))
