"""Independent formulations of a gate application, used to pin the oracle.

Neither function walks amplitude blocks the way the oracle does:

* ``tensor_apply`` views the statevector as an n-way tensor (axis of q_0 last,
  since q_0 is least significant, paper Sec. 2) and contracts U with the target
  axes via ``numpy.tensordot``; controls are handled by slicing the tensor at the
  control values (paper Sec. 2.4: the gate acts only where the controls hold).
* ``kron_operator`` builds the full D x D operator from Kronecker products (the
  tensor-product route the paper's method avoids, Sec. 1/2.5), with q_0 as the
  right-most factor: G = ... (x) U (x) ... (x) I_{d_0}; with controls,
  G = P_v (x) U + (I - P_v (x) I), P_v the projector onto the control values.
  It handles targets that are adjacent positions listed in ascending order.
"""
from functools import reduce

import numpy as np


def tensor_apply(dims, psi, targets, U, controls=(), values=()):
    n = len(dims)
    T = np.array(psi, dtype=np.complex128).reshape(tuple(reversed(dims)))
    ax = {q: n - 1 - q for q in range(n)}
    idx = [slice(None)] * n
    for c, v in zip(controls, values):
        idx[ax[c]] = int(v)
    idx = tuple(idx)
    sub = T[idx]
    remaining = [q for q in reversed(range(n)) if q not in controls]
    sub_ax = {q: i for i, q in enumerate(remaining)}
    k = len(targets)
    tdims = [dims[t] for t in targets]
    # Local index a = sum_l a_l prod_{l'<l} d_{t_l'}: in C order the last axis is t_0.
    Ut = np.asarray(U, dtype=np.complex128).reshape(tuple(reversed(tdims)) * 2)
    tgt_axes = [sub_ax[t] for t in reversed(targets)]
    R = np.tensordot(Ut, sub, axes=(list(range(k, 2 * k)), tgt_axes))
    R = np.moveaxis(R, list(range(k)), tgt_axes)
    T[idx] = R
    return T.reshape(-1)


def kron_operator(dims, targets, U, controls=(), values=()):
    n = len(dims)
    k = len(targets)
    t0 = targets[0]
    assert list(targets) == list(range(t0, t0 + k)), "targets must be adjacent and ascending"
    M = int(np.prod([dims[t] for t in targets]))
    cv = dict(zip(controls, values))

    def build(with_u: bool, project: bool):
        ops = []
        q = n - 1
        while q >= 0:
            if q == t0 + k - 1:
                ops.append(np.asarray(U, dtype=np.complex128) if with_u else np.eye(M))
                q -= k
                continue
            if project and q in cv:
                P = np.zeros((dims[q], dims[q]))
                P[cv[q], cv[q]] = 1.0
                ops.append(P)
            else:
                ops.append(np.eye(dims[q]))
            q -= 1
        return reduce(np.kron, ops)

    if not controls:
        return build(True, False)
    D = int(np.prod(dims))
    return build(True, True) + (np.eye(D) - build(False, True))
