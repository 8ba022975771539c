"""Continuous-batching server: results are the same alone and in the mix, the
HBM budget is respected, and requests that arrive while others are on the GPU
join them before those finish."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_close
from qd_inputs import circuits

pytestmark = pytest.mark.gpu


def qd():
    import paper_2410_17876_amd as q
    return q


def make_requests(count, qps, lo, hi, depth_lo, depth_hi, seed):
    reqs = circuits.served_requests(qps=qps, count=count, seed=seed, lo=lo, hi=hi, depth_lo=depth_lo,
                                    depth_hi=depth_hi)
    return reqs, qd().serve.requests_from_specs(reqs)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_served_results_equal_alone_and_oracle(precision):
    specs, reqs = make_requests(40, qps=400.0, lo=1e3, hi=2e5, depth_lo=20, depth_hi=120, seed=31)
    srv = qd().serve.Server(precision, budget_bytes=50e9, quantum=16, keep_states=True)
    rep = srv.run(reqs, realtime=True)
    assert rep["requests"] == 40 and rep["rejected"] == 0
    assert rep["max_resident_requests"] > 1
    for r, sp in zip(sorted(srv.finished, key=lambda r: r.rid), specs):
        alone = qd().State(sp.spec.dims, precision)
        alone.run_circuit(sp.spec.gates())
        got = r.state.amplitudes()
        assert np.array_equal(got, alone.amplitudes()), f"request {r.rid} differs from its solo run"
        assert abs(r.norm - 1.0) < (1e-12 if precision == "c128" else 1e-4)
        if sp.spec.D <= 20000:
            assert_close(got, oracle.run(sp.spec.dims, sp.spec.gates()), precision, f"request {r.rid}")
        alone.close()
    srv.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_served_with_lookahead_matches_oracle(precision):
    # ticks planned with a commuting look-ahead: the order within each quantum
    # changes, the state agrees with the in-order one up to rounding
    specs, reqs = make_requests(24, qps=400.0, lo=1e3, hi=2e4, depth_lo=40, depth_hi=160, seed=33)
    srv = qd().serve.Server(precision, budget_bytes=50e9, quantum=16, keep_states=True, reorder=64)
    rep = srv.run(reqs, realtime=True)
    assert rep["requests"] == 24 and rep["rejected"] == 0
    for r, sp in zip(sorted(srv.finished, key=lambda r: r.rid), specs):
        assert abs(r.norm - 1.0) < (1e-12 if precision == "c128" else 1e-4)
        assert_close(r.state.amplitudes(), oracle.run(sp.spec.dims, sp.spec.gates()), precision, f"request {r.rid}")
    srv.close()


def test_budget_is_respected_and_oversized_rejected():
    specs, reqs = make_requests(30, qps=1000.0, lo=1e4, hi=1e6, depth_lo=10, depth_hi=40, seed=32)
    biggest = max(r.D for r in reqs) * 8
    budget = 2.5 * biggest
    huge = qd().serve.ServeRequest(999, 0.0, [7] * 11, qd().GateList([]))  # 1.98e9 amps: over the budget
    srv = qd().serve.Server("c64", budget_bytes=budget, quantum=8)
    rep = srv.run(reqs + [huge], realtime=True)
    assert rep["rejected"] == 1 and huge.rejected
    assert rep["requests"] == 30
    assert srv.peak_bytes <= budget
    srv.close()


def test_arrivals_join_while_others_run():
    # a long request arrives first; short ones arrive while it runs and must be
    # admitted -- and finish -- before it does
    # (the long one: 2^27 amplitudes, 600 gates, 2 gates per tick -- about 300
    # ticks, far longer than the ~15 ms over which the short ones arrive)
    specs, reqs = make_requests(12, qps=1000.0, lo=1e3, hi=1e4, depth_lo=10, depth_hi=20, seed=33)
    long_spec = circuits.CircuitSpec([2] * 27, 600, 77)
    long_req = qd().serve.ServeRequest(100, 0.0, long_spec.dims, qd().GateList(long_spec.gates()))
    for r in reqs:
        r.arrival += 0.005
    srv = qd().serve.Server("c64", quantum=2)
    srv.run([long_req] + reqs, realtime=True)
    shorts = [r for r in srv.finished if r.rid != 100]
    assert all(r.admitted < long_req.finished for r in shorts)
    assert sum(r.finished < long_req.finished for r in shorts) >= len(shorts) // 2
    srv.close()


def test_empty_circuit_retires_and_norms_match():
    # A request with no gates finishes at the next tick with the norm of
    # |0...0>; every served norm (written by the device into pinned memory, with
    # no wait on the shared stream) equals qd_norm of the final state bitwise.
    specs, reqs = make_requests(10, qps=2000.0, lo=1e3, hi=1e5, depth_lo=5, depth_hi=30, seed=34)
    empty = qd().serve.ServeRequest(500, 0.001, [3, 2, 5], qd().GateList([]))
    srv = qd().serve.Server("c128", quantum=4, keep_states=True)
    rep = srv.run(reqs + [empty], realtime=True, timeout=60.0)
    assert rep["requests"] == 11
    assert empty.finished is not None and empty.norm == 1.0
    for r in srv.finished:
        assert r.norm == r.state.norm(), f"request {r.rid}"
    srv.close()
