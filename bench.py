#!/usr/bin/env python3
"""Benchmark of block-simulation gate application on one MI355X.

Workload: the mixed-radix register 2^14 x 3^8 x 4^2 (D = 1.72e9 amplitudes;
q_0..q_13 qubits, q_14..q_21 qutrits, q_22..q_23 ququads), a normalised complex
Gaussian initial state (seed 1001) resident in HBM, and a 500-gate circuit: w.p.
0.1 a 2-qudit Haar unitary, else the basic mix (1-qudit Haar 60%, DFT/X/Z 20%,
controlled X 20%). One step = the whole circuit applied once, then the FP64
norm. Six runs of the same circuit:

  lookahead c128  qd_apply_circuit with LDS-staged fusion and a 256-gate
                  commuting look-ahead (a pass also takes later gates that
                  commute with the ones it skips) -- the headline `value`
  fused c128      the same passes strictly in the given order (the library's
                  default circuit path)
  plain c128      one sweep per gate (qd_apply_gate)
  the same three in c64

Metric: gate-amplitude updates/s = sum over gates of the amplitudes each gate
changes (identity rows of U skipped; only classes whose controls hold) / wall
time of the timed steps. It counts per original gate, so fusion raises it
without moving more bytes.

Roofline: for the kernel instantiation with the largest total time, the bytes
it must move per launch (plain sweep: 2 x changed amplitudes x bytes; fused
pass: 2 x D x bytes, one read and one write of the whole state) / its average
launch time, measured with HIP events around every launch on the stream the
kernels run on, against 8 TB/s. `traffic` is the counter-measured HBM bytes per
launch (profiles/*traffic*.json, when taken for the current kernel source).

Also reported: the in-place read+rewrite copy ceiling measured on the same
buffer (qd_copy_ceiling), and the FP64 oracle (one thread) on the first gates
of the same circuit and state as the CPU baseline. Further runs under `runs`:
the 12-ququint workload (300 Haar gates of 25 and 125 members, MFMA) in
complex64 and complex128, the 512-circuit batched workload, the sparse GHZ
builds and the served workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PEAK_MFMA_TFLOPS = {"c64": 157.3, "c128": 78.6}  # dense FP32 / FP64 matrix peaks
# vector FMA peaks: 256 CUs x 2.4 GHz x 256 (FP32) or 128 (FP64) flops per clock per CU
PEAK_VALU_TFLOPS = {"c64": 157.3, "c128": 78.6}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_key(info: dict, precision: str) -> str:
    t = "double" if precision == "c128" else "float"
    if info["kernel"] == "sweep_monomial":
        a = info["updated"] // max(1, info["classes"])
        return f"sweep_monomial<{t},A={a}>"
    if info["kernel"] == "identity":
        return "identity"
    return f"{info['kernel']}<{t},M={info['M']}>"


# The sources each kernel family (and the planner that shapes its launches) is
# built from: counter readings stay valid while these files are unchanged.
KERNEL_SOURCES = {
    "fused_tile": ["fused.hip", "fused.h", "device.h", "plan.h", "kernels.h", "fusion.cpp", "fusion.h"],
    "batch_tile": ["fused.hip", "fused.h", "device.h", "plan.h", "kernels.h", "fusion.cpp", "fusion.h", "abi.cpp"],
    "sweep": ["sweep.hip", "device.h", "plan.h", "kernels.h", "planner.cpp", "planner.h"],
    "block_mfma": ["mfma.hip", "device.h", "plan.h", "kernels.h", "planner.cpp", "planner.h"],
}


def source_digest(kernel: str) -> str:
    fam = next((k for k in KERNEL_SOURCES if kernel.startswith(k)), None)
    names = KERNEL_SOURCES[fam] if fam else sorted(os.listdir(os.path.join(ROOT, "paper_2410_17876_amd", "csrc")))
    h = hashlib.sha256()
    for name in names:
        h.update(name.encode())
        h.update(open(os.path.join(ROOT, "paper_2410_17876_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Counter-measured bytes per launch for `kernel`, if taken on its current sources."""
    digest = source_digest(kernel)
    for f in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.json")):
        try:
            d = json.load(open(f))
        except Exception:
            continue
        if d.get("kernel") == kernel and d.get("source_digest") == digest:
            return d.get("bytes_per_launch")
    return None


TILE = {"c128": 0, "c64": 0}
MIN_RUN = {"c128": 0, "c64": 0}
# Look-ahead of the planner in "lookahead" mode: a pass also takes later gates
# that commute with the ones it skips (qd_circuit_options.reorder).
LOOKAHEAD = 256


def build_units(qd, dims, gates, precision, mode):
    """The launches of one step: (key, bytes per launch, updates, callable)."""
    D = math.prod(dims)
    ab = 16 if precision == "c128" else 8
    infos = [qd.gate_info(dims, g.targets, g.U, g.controls, g.values, precision) for g in gates]
    units = []
    if mode == "plain":
        for g, info in zip(gates, infos):
            if info["kernel"] == "identity":
                continue
            units.append((kernel_key(info, precision), info["bytes"], info["updated"], ("gate", g), info["flops"]))
        return units
    reorder = LOOKAHEAD if mode == "lookahead" else 0  # LOOKAHEAD: set from --lookahead
    plan, order = qd.circuit_plan(dims, gates, precision, tile_amps=TILE[precision], min_run=MIN_RUN[precision],
                                  reorder=reorder,
                                  with_order=True)
    live = [i for i, info in enumerate(infos) if info["kernel"] != "identity"]
    assert sorted(order) == live
    pos = 0
    for ngates, tile in plan:
        idx = order[pos:pos + ngates]  # each pass's gates in the planned order
        pos += ngates
        upd = sum(infos[i]["updated"] for i in idx)
        if tile:
            t = "double" if precision == "c128" else "float"
            units.append((f"fused_tile<{t}>", 2 * D * ab, upd, ("pass", qd.GateList([gates[i] for i in idx])),
                          sum(infos[i]["flops"] for i in idx)))
        else:
            i = idx[0]
            units.append((kernel_key(infos[i], precision), infos[i]["bytes"], upd, ("gate", gates[i]),
                          infos[i]["flops"]))
    assert pos == len(live)
    return units


def run_mode(qd, st, dims, gates, precision, mode, steps, warmup):
    import torch

    units = build_units(qd, dims, gates, precision, mode)
    stream = st.stream

    def step(events=None):
        for u, (_, _, _, (kind, obj), _) in enumerate(units):
            if events is not None:
                events[u][0].record(stream)
            if kind == "gate":
                st.apply_gate(obj)
            else:
                st.run_circuit(obj, fuse=True, tile_amps=TILE[precision], min_run=MIN_RUN[precision])
            if events is not None:
                events[u][1].record(stream)
        return st.norm()

    for w in range(warmup):
        nrm = step()
        log(f"{mode} {precision}: warmup step {w} done, norm {nrm:.15f}")
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in units]
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = [step(evs[k]) for k in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{mode} {precision}: {steps} timed steps in {wall:.3f} s ({len(units)} launches per step), "
        f"norms {[round(x, 12) for x in norms]}")

    per = {}
    for k in range(steps):
        for u, (key, nbytes, _, _, flops) in enumerate(units):
            e = per.setdefault(key, {"launches": 0, "ms": 0.0, "bytes": 0, "flops": 0})
            e["launches"] += 1
            e["ms"] += evs[k][u][0].elapsed_time(evs[k][u][1])
            e["bytes"] += nbytes
            e["flops"] += flops
    updates = steps * sum(u[2] for u in units)
    kernels = {key: {"launches": e["launches"], "avg_us": round(1e3 * e["ms"] / e["launches"], 2),
                     "total_ms": round(e["ms"], 3),
                     "GBps": round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1) if e["ms"] > 0 else None,
                     "TFLOPs": round(e["flops"] / (e["ms"] * 1e-3) / 1e12, 2) if e["ms"] > 0 else None}
               for key, e in per.items()}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = per[dom]
    if dom.startswith("block_mfma"):
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        peak = PEAK_MFMA_TFLOPS[precision]
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": load_traffic(dom), "kernel": dom,
                "avg_us": kernels[dom]["avg_us"], "flops_per_launch": d["flops"] // d["launches"],
                "bytes_per_launch": d["bytes"] // d["launches"]}
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        alu = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": load_traffic(dom), "kernel": dom,
                "avg_us": kernels[dom]["avg_us"], "bytes_per_launch": d["bytes"] // d["launches"],
                # the same launches against the vector ALU: the gates' useful flops (8 M per
                # changed amplitude, dense gates) per second over the FP64 / FP32 vector peak
                "alu_tflops": round(alu, 2), "alu_peak_tflops": PEAK_VALU_TFLOPS[precision],
                "alu_frac": round(alu / PEAK_VALU_TFLOPS[precision], 4),
                "flops_per_launch": d["flops"] // d["launches"]}
    return {
        "value": updates / wall,
        "ms_per_step": 1e3 * wall / steps,
        "launches_per_step": len(units),
        "updates_per_step": updates // steps,
        "norm_last_step": norms[-1],
        "roofline": roof,
        "kernels": kernels,
    }


def lookahead_roundtrip(qd, st, dims, gates, precision, upload, values_at):
    """The look-ahead path on the full register: the circuit, then its inverse
    (each through qd_apply_circuit with the same look-ahead), must return the
    input; max-abs and relative error on sampled amplitudes."""
    import numpy as np

    upload(st)
    st.run_circuit(gates, reorder=LOOKAHEAD)
    st.run_circuit([g.inverse() for g in reversed(gates)], reorder=LOOKAHEAD)
    st.synchronize()
    rng = np.random.default_rng(45)
    idx = np.unique(np.concatenate([rng.integers(0, st.D, size=20000), [0, st.D - 1]]))
    t = __import__("torch").as_tensor(idx, device=st.device)
    v = st.buffer.view(-1, 2)[t].double().cpu().numpy()
    got = v[:, 0] + 1j * v[:, 1]
    want = values_at(idx)
    if precision == "c64":
        want = round32(want)
    err = error_stats(got, want)
    log(f"{precision}: look-ahead circuit + inverse on the full register: max-abs error {err['max_abs']:.3e} "
        f"on {idx.size} sampled amplitudes")
    return dict(err, samples=int(idx.size), gates=2 * len(gates))


def run_precision(qd, dims, gates, precision, upload, steps, warmup, modes, values_at=None):
    import torch

    st = qd.State(dims, precision, init=None)
    ab = 16 if precision == "c128" else 8
    best_ms = st.copy_ceiling(3)
    ceiling = 2 * st.D * ab / (best_ms * 1e-3) / 1e9
    log(f"{precision}: copy ceiling {ceiling:.1f} GB/s ({best_ms:.3f} ms per read+rewrite pass)")
    out = {"copy_ceiling_GBps": round(ceiling, 1)}
    for mode in modes:
        t0 = time.time()
        upload(st)
        st.synchronize()
        log(f"{precision}: state uploaded in {time.time() - t0:.1f} s")
        out[mode] = run_mode(qd, st, dims, gates, precision, mode, steps, warmup)
    if "lookahead" in modes and values_at is not None:
        out["lookahead"]["roundtrip"] = lookahead_roundtrip(qd, st, dims, gates, precision, upload, values_at)
    st.close()
    del st
    torch.cuda.empty_cache()
    return out


def run_batched(qd, precision, steps, warmup, tune_cache, lookahead):
    """The batched workload: 512 independent circuits (6..16 qudits, d in 2..5,
    D <= 1e6, depth 100..1000, |0..0>) advanced together by qd_batch_apply,
    passes planned with the given commuting look-ahead."""
    import torch
    from qd_inputs import circuits

    specs = circuits.batched_specs()
    t0 = time.time()
    lists = [qd.GateList(s.gates()) for s in specs]
    log(f"batched {precision}: {len(specs)} circuits generated in {time.time() - t0:.1f} s "
        f"(sum D = {sum(s.D for s in specs)}, gates = {sum(len(g) for g in lists)})")
    # Autotune the tile shape on a sample: 64 circuits, first 100 gates each,
    # timing graph replays of a compiled plan per candidate (what the timed run
    # does); the tuner's untimed warm-up call of each candidate compiles it.
    sample = qd.batch.BatchRunner([s.dims for s in specs[:64]], precision)
    sample_lists = [qd.GateList(g.gates[:100]) for g in lists[:64]]
    sample_plans = {}

    def trial(tile, run_len):
        if (tile, run_len) not in sample_plans:
            sample_plans[(tile, run_len)] = sample.compile(sample_lists, tile_amps=tile, min_run=run_len,
                                                           reorder=lookahead)
        sample_plans[(tile, run_len)].run(graph=True)
        torch.cuda.synchronize()

    tuned = qd.tune.tune(trial, precision, f"batched-workload-v3-lookahead{lookahead}", tune_cache)
    for p in sample_plans.values():
        p.close()
    sample.close()
    tile, run_len = tuned["tile_amps"], tuned["min_run"]
    log(f"batched {precision}: autotuned tile {tile}, min run {run_len} ({'cached' if tuned['cached'] else 'measured'})")
    runner = qd.batch.BatchRunner([s.dims for s in specs], precision)
    ab = 16 if precision == "c128" else 8
    updates = 0
    flops = 0
    pass_bytes = 0
    for s, gl in zip(specs, lists):
        infos = [qd.gate_info(s.dims, g.targets, g.U, g.controls, g.values, precision) for g in gl.gates]
        updates += sum(i["updated"] for i in infos)
        flops += sum(i["flops"] for i in infos)
        npass = len(qd.circuit_plan(s.dims, gl, precision, tile_amps=tile, min_run=run_len, reorder=lookahead))
        pass_bytes += npass * 2 * s.D * ab
    t0 = time.time()
    plan = runner.compile(lists, tile_amps=tile, min_run=run_len, reorder=lookahead)
    log(f"batched {precision}: compiled {plan.rounds} rounds, {plan.items} items in {time.time() - t0:.1f} s")
    timing = {}
    for mode in ("eager", "graph"):
        for w in range(warmup):
            plan.run(graph=(mode == "graph"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run(graph=(mode == "graph"))
        torch.cuda.synchronize()
        timing[mode] = time.perf_counter() - t0
        log(f"batched {precision}: {steps} timed steps ({mode} replay) in {timing[mode]:.3f} s")
    wall = timing["graph"]
    norms = [st.norm() for st in runner.states[:8]]
    rounds, items = plan.rounds, plan.items
    plan.close()
    runner.close()
    torch.cuda.empty_cache()
    log(f"batched {precision}: norms of the first states {norms[:3]}")
    achieved = pass_bytes * steps / wall / 1e9
    alu = flops * steps / wall / 1e12
    return {"value": updates * steps / wall, "unit": "updates/s", "dtype": "f64" if precision == "c128" else "f32",
            "ms_per_step": 1e3 * wall / steps, "ms_per_step_eager_launches": 1e3 * timing["eager"] / steps,
            "launch_rounds_per_step": rounds, "items_per_step": items,
            "path": "compiled batch replayed as one hipGraph per step",
            "lookahead": lookahead,
            "autotuned": {"tile_amps": tile, "min_run": run_len, "timings_s": tuned.get("timings_s")},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                         "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None, "kernel": "batch_tile",
                         # the same run against the vector ALU: the gates' useful flops
                         # (8 M per changed amplitude, dense gates) over the FP64 / FP32 vector peak
                         "alu_tflops": round(alu, 2), "alu_peak_tflops": PEAK_VALU_TFLOPS[precision],
                         "alu_frac": round(alu / PEAK_VALU_TFLOPS[precision], 4),
                         "note": "whole-run averages over all rounds: 2 x D x bytes per (state, pass); "
                                 "the gates' useful flops"}}


def run_served(qd, n_closed, n_open, loads, lookahead):
    """The served workload: requests with log-uniform sizes in [1e3, 1e8]
    amplitudes (d in 2..7), depth 50..500 of the basic mix, complex64, admitted
    under a 200 GB HBM budget. First the closed-loop capacity (all requests
    present at t = 0), then open-loop Poisson arrivals at each of `loads` x
    capacity. One request stream is generated (at rate 1/s) and reused: Poisson
    arrivals at rate q are the rate-1 arrival times divided by q. Every tick's
    passes use the given commuting look-ahead."""
    import torch
    from qd_inputs import circuits

    t0 = time.time()
    n = max(n_closed, n_open)
    specs = circuits.served_requests(qps=1.0, count=n)
    base = qd.serve.requests_from_specs(specs)
    log(f"served: {n} requests generated in {time.time() - t0:.1f} s "
        f"(sum D = {sum(r.D for r in base):.3g}, gates = {sum(len(r.gates) for r in base)})")

    def fresh(count, rate):
        return [qd.serve.ServeRequest(r.rid, r.arrival / rate if rate else 0.0, r.dims, r.gates) for r in base[:count]]

    upd = lambda reqs: sum(qd.gate_info(r.dims, g.targets, g.U, g.controls, g.values, "c64")["updated"]
                           for r in reqs for g in r.gates.gates)
    srv = qd.serve.Server("c64", budget_bytes=200e9, quantum=32, reorder=lookahead)
    srv.run(fresh(16, 0), realtime=False)  # warm-up
    srv.close()
    closed = fresh(n_closed, 0)
    srv = qd.serve.Server("c64", budget_bytes=200e9, quantum=32, reorder=lookahead)
    rc = srv.run(closed, realtime=False)
    srv.close()
    cap = rc["throughput_rps"]
    log(f"served: closed-loop capacity {cap:.1f} requests/s ({rc['wall_s']:.2f} s for {n_closed})")
    opened = {}
    for load in loads:
        reqs = fresh(n_open, load * cap)
        srv = qd.serve.Server("c64", budget_bytes=200e9, quantum=32, reorder=lookahead)
        ro = srv.run(reqs, realtime=True)
        srv.close()
        ro = dict(ro, offered_rps=load * cap, load=load, updates_per_s=upd(reqs) / ro["wall_s"])
        opened[f"{load:.2f}"] = ro
        log(f"served: open loop at {load:.2f} x capacity: p50 {ro['p50_ms']:.1f} ms, p99 {ro['p99_ms']:.1f} ms")
    torch.cuda.empty_cache()
    main = opened[f"{loads[len(loads) // 2]:.2f}"]
    return {"workload": "Poisson arrivals, sizes log-uniform 1e3..1e8 amplitudes (d in 2..7), depth 50..500, "
                        "basic gate mix, complex64, 200 GB HBM budget (seed 1003)",
            "value": main["updates_per_s"], "unit": "updates/s", "dtype": "f32",
            "closed_loop": {"requests": n_closed, "capacity_rps": cap, "wall_s": rc["wall_s"],
                            "updates_per_s": upd(closed) / rc["wall_s"], "p50_ms": rc["p50_ms"],
                            "p99_ms": rc["p99_ms"]},
            "open_loop": opened,
            "latency": "arrival -> final state resident and its FP64 norm returned to the host",
            "lookahead": lookahead}


GHZ_REGISTERS = ((2, 62), (3, 39), (4, 31), (5, 27))
# past the paper's signed 64-bit index (multi-word keys)
GHZ_WIDE_REGISTERS = ((2, 100), (3, 63), (4, 50), (5, 43), (7, 45))


def ghz_gates(d, n):
    from qd_inputs import Gate, dft, shift
    return [Gate((0,), dft(d))] + [Gate((q,), shift(d, v), (0,), (v,)) for q in range(1, n) for v in range(1, d)]


def cpu_baseline_sparse():
    """The sparse oracle (plain Python, one thread) on the same GHZ builds, in ms."""
    from oracle import sparse as soracle
    out = {}
    for d, n in GHZ_REGISTERS + GHZ_WIDE_REGISTERS:
        t0 = time.perf_counter()
        soracle.run([d] * n, ghz_gates(d, n))
        out[f"{d}^{n}"] = round(1e3 * (time.perf_counter() - t0), 3)
    return out


def run_sparse_ghz(qd, reps=3):
    """The sparse variant on the paper's GHZ registers: GHZ_d on 62 qubits, 39
    qutrits, 31 ququads and 27 ququints (DFT on q0, then X_{+v} on each other
    qudit controlled on q0 = v), from |0...0>."""
    out = {}
    for d, n in GHZ_REGISTERS + GHZ_WIDE_REGISTERS:
        gl = qd.GateList(ghz_gates(d, n))  # marshalled once, outside the timed region
        gates = gl.gates
        best = None
        for rep in range(reps + 1):  # the first build warms up
            st = qd.SparseState([d] * n)
            torch_sync()
            t0 = time.perf_counter()
            st.run(gl)  # qd_sparse_apply_circuit
            nnz = st.nnz()  # waits for the state's stream
            dt = time.perf_counter() - t0
            words = st.words
            st.close()
            if rep and (best is None or dt < best):
                best = dt
        out[f"{d}^{n}"] = {"gates": len(gates), "nnz": nnz, "key_words": words, "ms": round(1e3 * best, 3),
                           "gates_per_s": round(len(gates) / best, 1)}
        log(f"sparse GHZ_{d} on {n} qudits ({words} key words): {len(gates)} gates in {1e3 * best:.3f} ms")
    return {"workload": "GHZ_d from |0...0> on 62 qubits, 39 qutrits, 31 ququads, 27 ququints (the paper's largest), "
                        "and past 2^64: 100 qubits, 63 qutrits, 50 ququads, 43 ququints, 45 qudits of dim 7 "
                        "(sparse, complex128)",
            "path": "qd_sparse_apply_circuit: one workgroup per gate (group by class in LDS, U x per class, keep "
                    "nonzeros, order by rank), enqueued with no host synchronisation; time = the call to the "
                    "entry count read back",
            "registers": out}


def torch_sync():
    import torch
    torch.cuda.synchronize()


def host_info() -> dict:
    """CPU model, usable cores and RAM of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram = round(int(line.split()[1]) * 1024 / 2**30, 1)
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return {"cpu_model": model, "cores": cores, "ram_GiB": ram}


def oracle_threads_all() -> int:
    # the host's usable cores, capped at the 16 a one-GPU share of the box has
    return max(1, min(16, host_info()["cores"]))


def cpu_baseline(qd, dims, gates, psi, seconds):
    """The FP64 oracle on the same circuit and state: one thread for about
    `seconds`, then the same gates on every usable core (OpenMP over classes,
    per-amplitude arithmetic unchanged)."""
    import oracle

    def leg(threads, max_gates=None):
        done, updates = 0, 0
        t0 = time.perf_counter()
        with oracle.threads(threads):
            for g in gates[:max_gates]:
                oracle.apply_gate(dims, psi, g)
                done += 1
                updates += qd.gate_info(dims, g.targets, g.U, g.controls, g.values, "c128")["updated"]
                if max_gates is None and time.perf_counter() - t0 >= seconds:
                    break
        return done, updates, time.perf_counter() - t0

    n1, u1, t1 = leg(1)
    nt = oracle_threads_all()
    nn, un, tn = leg(nt, n1)
    host = host_info()
    return {"value": un / tn, "unit": "updates/s", "cores": nt, "kind": "oracle",
            "sample": f"first {nn} of {len(gates)} gates on the full D={math.prod(dims)} state "
                      f"(FP64 oracle, {nt} threads, {tn:.1f} s; one thread: {t1:.1f} s)",
            "single_core": {"value": u1 / t1, "unit": "updates/s", "cores": 1, "gates": n1, "seconds": round(t1, 2)},
            "all_cores": {"value": un / tn, "unit": "updates/s", "cores": nt, "gates": nn, "seconds": round(tn, 2)},
            "host": host}


def round32(v):
    import numpy as np
    return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)


def error_stats(got, ref) -> dict:
    import numpy as np
    d = np.abs(got - ref)
    mx = float(np.max(d))
    return {"max_abs": mx, "rel_to_max_amp": mx / float(np.max(np.abs(ref))),
            "rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}


def headline_error_vs_oracle(qd, gates_fn, lookahead):
    """The headline path (qd_apply_circuit, fused passes, the same look-ahead and
    default tiles) on the scaled-down register 2^10 x 3^6 x 4^2 with the same
    500-gate mix and a Gaussian input, compared element by element with the FP64
    oracle (the complex64 run against the oracle from the FP32-rounded input)."""
    import numpy as np
    import oracle
    from qd_inputs import states

    dims = [2] * 10 + [3] * 6 + [4] * 2
    _, gates = gates_fn(dims)
    D = math.prod(dims)
    psi0 = states.GaussianState(D, seed=1001).full()
    out = {"register": "2^10 x 3^6 x 4^2", "D": D, "gates": len(gates), "lookahead": lookahead}
    t0 = time.perf_counter()
    for p in ("c128", "c64"):
        inp = psi0 if p == "c128" else round32(psi0)
        with oracle.threads(oracle_threads_all()):
            ref = oracle.run(dims, gates, inp)
        st = qd.State(dims, p, init=None).set_amplitudes(psi0)
        st.run_circuit(gates, reorder=lookahead)
        out[p] = error_stats(st.amplitudes(), ref)
        st.close()
    log(f"headline path vs oracle on {out['register']}: c128 max-abs {out['c128']['max_abs']:.3e}, "
        f"c64 max-abs {out['c64']['max_abs']:.3e} ({time.perf_counter() - t0:.1f} s)")
    return out


def run_plain_small(qd, reps):
    """The plain workload: dims [2,2,2,2,3,3] (D = 144), complex128, |0..0>, 200
    gates of the basic mix (seed 1000). Launch-latency bound: one launch per
    gate (qd_apply_gate) against the whole circuit in one fused launch
    (qd_apply_circuit). Error vs the FP64 oracle on the whole state."""
    import oracle
    import torch
    from qd_inputs import circuits

    dims, gates = circuits.plain()
    gl = qd.GateList(gates)
    ref = oracle.run(dims, gates)
    upd = sum(qd.gate_info(dims, g.targets, g.U, g.controls, g.values, "c128")["updated"] for g in gates)
    out = {"workload": "dims [2,2,2,2,3,3] (D=144), complex128, |0..0>, 200 gates of the basic mix (seed 1000)",
           "unit": "gates/s", "dtype": "f64"}
    st = qd.State(dims, "c128")
    forms = {"per_gate_launches": lambda: st.run(gates),
             "one_launch": lambda: st.run_circuit(gl)}
    for name, fn in forms.items():
        st.reset(0)
        info = fn()
        err = error_stats(st.amplitudes(), ref)
        for _ in range(max(1, reps // 10)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = {"value": len(gates) * reps / dt, "unit": "gates/s", "updates_per_s": upd * reps / dt,
             "us_per_circuit": 1e6 * dt / reps, "circuits": reps, "error_vs_oracle": err}
        if name == "one_launch":
            r["passes"] = info["passes"]
            r["fused_passes"] = info["fused_passes"]
        out[name] = r
        log(f"plain D=144 {name}: {r['value']:.3e} gates/s ({r['us_per_circuit']:.1f} us per 200-gate circuit), "
            f"max-abs error {err['max_abs']:.2e}")
    out["value"] = out["one_launch"]["value"]
    st.close()
    return out


def ququint_layer_errors(qd):
    """The ququint gate mix (Haar gates on 2 or 3 of the qudits, 25 and 125
    members) on 8 ququints (D = 390625, the largest the oracle advances in a few
    seconds per layer), GPU and oracle in lockstep from |0..0>: the max-abs error
    after each gate (a layer: the state is materialised after every gate on this
    path), in complex64 and complex128."""
    import numpy as np
    import oracle
    from qd_inputs import circuits

    dims, gates = circuits.fused(dims=[5] * 8)
    ref = oracle.zero_state(dims)
    sts = {p: qd.State(dims, p) for p in ("c64", "c128")}
    errs = {p: [] for p in sts}
    t0 = time.perf_counter()
    with oracle.threads(oracle_threads_all()):
        for g in gates:
            oracle.apply_gate(dims, ref, g)
            for p, st in sts.items():
                st.apply_gate(g)
                errs[p].append(float(np.max(np.abs(st.amplitudes() - ref))))
    for st in sts.values():
        st.close()
    log(f"ququint 5^8 lockstep, {len(gates)} layers in {time.perf_counter() - t0:.1f} s: max-abs error "
        f"c64 {max(errs['c64']):.2e}, c128 {max(errs['c128']):.2e}")
    return {"register": "5^8 (D=390625)", "gates": len(gates), "seed": circuits.SEEDS["fused"],
            "layer": "one gate (the GPU materialises the state after every gate)",
            "c64_max_abs": max(errs["c64"]), "c128_max_abs": max(errs["c128"]),
            "c64_per_layer": [float(f"{e:.3g}") for e in errs["c64"]],
            "c128_per_layer": [float(f"{e:.3g}") for e in errs["c128"]]}


def main() -> int:
    global LOOKAHEAD
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--gates", type=int, default=500)
    ap.add_argument("--modes", default="lookahead,fused,plain",
                    help="comma list of lookahead (fused passes, commuting look-ahead), fused (in order), plain")
    ap.add_argument("--lookahead", type=int, default=LOOKAHEAD,
                    help="look-ahead in gates for lookahead mode and the batched runs (0 = in order)")
    ap.add_argument("--no-c64", action="store_true", help="skip the complex64 runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ququint", action="store_true", help="skip the 12-ququint MFMA workloads")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse GHZ builds")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-circuit batched workload")
    ap.add_argument("--no-served", action="store_true", help="skip the served (continuous batching) workload")
    ap.add_argument("--served-closed", type=int, default=600,
                    help="requests in the closed-loop capacity run (the same stream as the open-loop runs)")
    ap.add_argument("--served-open", type=int, default=600, help="requests in each open-loop run")
    ap.add_argument("--served-loads", default="0.5,0.8,0.95",
                    help="open-loop loads as fractions of the closed-loop capacity")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "gpurun_out", "tune_cache.json"),
                    help="autotuner cache file")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-error", action="store_true",
                    help="skip the error checks against the oracle (headline path on 2^10 x 3^6 x 4^2, ququint layers)")
    ap.add_argument("--no-plain-small", action="store_true", help="skip the D=144 launch-latency workload")
    ap.add_argument("--plain-small-reps", type=int, default=2000, help="circuits timed per form on D=144")
    ap.add_argument("--small", action="store_true", help="2^10 x 3^6 x 4^2 register (quick check)")
    ap.add_argument("--tile-c128", type=int, default=0, help="fused tile size, c128 (0 = library default)")
    ap.add_argument("--tile-c64", type=int, default=0, help="fused tile size, c64 (0 = library default)")
    ap.add_argument("--min-run-c128", type=int, default=0,
                    help="contiguous run a fused tile must hold, c128 (0 = library default)")
    ap.add_argument("--min-run-c64", type=int, default=0,
                    help="contiguous run a fused tile must hold, c64 (0 = library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the sharded multi-GPU "
              "path is a design only).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    import paper_2410_17876_amd as qd
    from qd_inputs import circuits, states

    dims = [2] * 10 + [3] * 6 + [4] * 2 if args.small else circuits.LARGE_DIMS
    _, gates = circuits.large(n_gates=args.gates, dims=dims)
    D = math.prod(dims)
    G = states.GaussianState(D, seed=circuits.SEEDS["large"])
    modes = [m for m in args.modes.split(",") if m]
    TILE["c128"], TILE["c64"] = args.tile_c128, args.tile_c64
    MIN_RUN["c128"], MIN_RUN["c64"] = args.min_run_c128, args.min_run_c64
    LOOKAHEAD = args.lookahead
    t0 = time.time()
    host = None
    if not args.no_cpu_baseline:
        host = G.full()
        log(f"host copy of the initial state generated in {time.time() - t0:.1f} s")

    def upload(st):
        if host is not None:
            hv = host.view(np.float64)
            chunk = 1 << 24
            for s in range(0, D, chunk):
                c = min(chunk, D - s)
                st.set_interleaved(hv[2 * s: 2 * (s + c)], s)
        else:
            G.fill(lambda start, vals: st.set_interleaved(vals, start))

    values_at = (lambda idx: host[idx]) if host is not None else G.values
    res = {}
    if modes:  # an empty --modes runs only the other workloads (for profiling them alone)
        res["c128"] = run_precision(qd, dims, gates, "c128", upload, args.steps, args.warmup, modes, values_at)
        if not args.no_c64:
            res["c64"] = run_precision(qd, dims, gates, "c64", upload, args.steps, args.warmup, modes, values_at)
    if not args.no_error:
        res["error"] = headline_error_vs_oracle(qd, lambda d: circuits.large(n_gates=args.gates, dims=d),
                                                LOOKAHEAD)
    if not args.no_plain_small:
        res["plain_small"] = run_plain_small(qd, args.plain_small_reps)
    if not args.no_ququint:
        qdims, qgates = circuits.fused()
        qst = qd.State(qdims, "c64")
        log(f"ququint register: D = {qst.D}, {len(qgates)} Haar gates (25x25 and 125x125)")
        res["ququint"] = run_mode(qd, qst, qdims, qgates, "c64", "plain", args.steps, args.warmup)
        qst.close()
        del qst
        torch.cuda.empty_cache()
        qst = qd.State(qdims, "c128")
        res["ququint_c128"] = run_mode(qd, qst, qdims, qgates, "c128", "plain", args.steps, args.warmup)
        qst.close()
        del qst
        torch.cuda.empty_cache()
        if not args.no_error:
            res["ququint_layers"] = ququint_layer_errors(qd)
    if not args.no_batched:
        for p in (["c64", "c128"] if not args.no_c64 else ["c128"]):
            res[f"batched_{p}"] = run_batched(qd, p, args.steps, args.warmup, args.tune_cache, args.lookahead)
    if not args.no_sparse:
        res["sparse"] = run_sparse_ghz(qd)
    if not args.no_served:
        res["served"] = run_served(qd, args.served_closed, args.served_open,
                                   [float(x) for x in args.served_loads.split(",")], args.lookahead)
    cpu = None
    if host is not None:
        cpu = cpu_baseline(qd, dims, gates, host, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.3e} updates/s ({cpu['sample']})")
        if "sparse" in res:
            res["sparse"]["cpu_oracle_ms"] = cpu_baseline_sparse()

    if not modes:
        print(json.dumps({"metric": "gate-amplitude updates/s", "value": None, "note": "no large-register run",
                          "runs": {k: v for k, v in res.items()}}, default=str), flush=True)
        return 0
    head_mode = modes[0]
    h = res["c128"][head_mode]
    workload = (f"large: dims {'2^10 x 3^6 x 4^2' if args.small else '2^14 x 3^8 x 4^2'} (D={D}), complex128, "
                f"{len(gates)}-gate circuit (seed {circuits.SEEDS['large']}), Gaussian initial state in HBM, "
                f"{head_mode} path")
    line = {
        "metric": "gate-amplitude updates/s",
        "value": h["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "D": D, "gates": len(gates), "precision": "c128", "path": head_mode,
                   "lookahead": LOOKAHEAD if head_mode == "lookahead" else 0},
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "error_vs_oracle": dict(res["error"], full_register_roundtrip=h.get("roundtrip")) if "error" in res else None,
        "copy_ceiling_GBps": {p: res[p]["copy_ceiling_GBps"] for p in ("c128", "c64") if p in res},
        "norm_last_step": h["norm_last_step"],
        "launches_per_step": h["launches_per_step"],
        "kernels": h["kernels"],
        "runs": {},
    }
    if "ququint" in res:
        r = res["ququint"]
        line["runs"]["ququint_mfma_c64"] = {
            "workload": "12 ququints (D=5^12), complex64, 300 Haar gates on 2 or 3 qudits (seed 1004), |0..0>",
            "value": r["value"], "unit": "updates/s", "dtype": "f32", "ms_per_step": r["ms_per_step"],
            "launches_per_step": r["launches_per_step"], "roofline": r["roofline"],
            "norm_last_step": r["norm_last_step"], "kernels": r["kernels"]}
        if "ququint_layers" in res:
            line["runs"]["ququint_mfma_c64"]["error_per_layer"] = res["ququint_layers"]
    if "ququint_c128" in res:
        r = res["ququint_c128"]
        line["runs"]["ququint_mfma_c128"] = {
            "workload": "12 ququints (D=5^12), complex128, the same 300 Haar gates (seed 1004), |0..0>",
            "value": r["value"], "unit": "updates/s", "dtype": "f64", "ms_per_step": r["ms_per_step"],
            "launches_per_step": r["launches_per_step"], "roofline": r["roofline"],
            "norm_last_step": r["norm_last_step"], "kernels": r["kernels"]}
    if "plain_small" in res:
        line["runs"]["plain_d144_c128"] = res["plain_small"]
    if "sparse" in res:
        line["runs"]["sparse_ghz_c128"] = res["sparse"]
    if "served" in res:
        line["runs"]["served_c64"] = res["served"]
    for p in ("c64", "c128"):
        if f"batched_{p}" in res:
            line["runs"][f"batched_{p}"] = dict(
                res[f"batched_{p}"],
                workload="512 circuits, 6..16 qudits, d in 2..5, D <= 1e6, depth 100..1000 (seed 1002), |0..0>")
    for p in ("c128", "c64"):
        if p not in res:
            continue
        for m in modes:
            if p == "c128" and m == head_mode:
                continue
            r = res[p][m]
            line["runs"][f"{m}_{p}"] = {"value": r["value"], "unit": "updates/s", "roundtrip": r.get("roundtrip"),
                                        "dtype": "f64" if p == "c128" else "f32",
                                        "ms_per_step": r["ms_per_step"], "launches_per_step": r["launches_per_step"],
                                        "roofline": r["roofline"], "norm_last_step": r["norm_last_step"],
                                        "kernels": r["kernels"]}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
