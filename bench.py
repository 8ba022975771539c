#!/usr/bin/env python3
"""Benchmark of the block-simulation gate sweep on one MI355X.

Workload: the large mixed-radix register 2^14 x 3^8 x 4^2 (D = 1.72e9
amplitudes; q_0..q_13 qubits, q_14..q_21 qutrits, q_22..q_23 ququads), a
normalised complex Gaussian initial state (seed 1001) resident in HBM, and a
500-gate circuit: w.p. 0.1 a 2-qudit Haar unitary, else the basic mix (1-qudit
Haar 60%, DFT/X/Z 20%, controlled X 20%). One step = the whole circuit applied
once, followed by the FP64 norm reduction. The complex128 run is the headline;
the complex64 run of the same circuit is reported beside it.

Metric: gate-amplitude updates/s = sum over gates of the amplitudes each gate
reads and writes (identity rows of U skipped, only classes that satisfy the
controls) / wall time of the timed steps. Algorithmic bytes = 2 x updates x
bytes per amplitude.

Roofline: for the kernel instantiation with the largest total time, algorithmic
bytes of its launches / their summed durations, measured with HIP events around
every launch on the stream the kernels run on, against 8 TB/s.

CPU baseline: the FP64 oracle (single thread) on the same state and circuit,
timed on its first gates until about --cpu-seconds have passed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0


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


def run_precision(qd, dims, gates, precision, upload, steps, warmup):
    import torch

    infos = [qd.gate_info(dims, g.targets, g.U, g.controls, g.values, precision) for g in gates]
    keys = [kernel_key(i, precision) for i in infos]
    st = qd.State(dims, precision, init=None)
    t0 = time.time()
    upload(st)
    st.synchronize()
    log(f"{precision}: state of {st.D} amplitudes uploaded in {time.time() - t0:.1f} s")
    stream = st.stream

    def step(events=None):
        for gi, g in enumerate(gates):
            if events is not None:
                events[gi][0].record(stream)
            st.apply_gate(g)
            if events is not None:
                events[gi][1].record(stream)
        return st.norm()

    for w in range(warmup):
        nrm = step()
        log(f"{precision}: warmup step {w} done, norm {nrm:.15f}")
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in gates]
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = []
    for k in range(steps):
        norms.append(step(evs[k]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{precision}: {steps} timed steps in {wall:.3f} s, norms {[round(x, 12) for x in norms]}")

    per = {}
    for k in range(steps):
        for gi, info in enumerate(infos):
            ms = evs[k][gi][0].elapsed_time(evs[k][gi][1])
            e = per.setdefault(keys[gi], {"launches": 0, "ms": 0.0, "bytes": 0})
            e["launches"] += 1
            e["ms"] += ms
            e["bytes"] += info["bytes"]
    updates = steps * sum(i["updated"] for i in infos)
    bytes_total = steps * sum(i["bytes"] for i in infos)
    kernels = {}
    for key, e in per.items():
        if key == "identity":
            continue
        kernels[key] = {"launches": e["launches"], "avg_us": round(1e3 * e["ms"] / e["launches"], 2),
                        "total_ms": round(e["ms"], 3),
                        "GBps": round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1) if e["ms"] > 0 else None}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = per[dom]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out = {
        "value": updates / wall,
        "ms_per_step": 1e3 * wall / steps,
        "updates_per_step": updates // steps,
        "algorithmic_GBps": bytes_total / wall / 1e9,
        "norm_last_step": norms[-1],
        "dominant": dom,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None,
                     "kernel": dom, "avg_us": kernels[dom]["avg_us"],
                     "bytes_per_launch": d["bytes"] // d["launches"]},
        "kernels": kernels,
    }
    st.close()
    del st
    torch.cuda.empty_cache()
    return out


def cpu_baseline(dims, gates, psi, infos, seconds):
    import oracle

    done, updates = 0, 0
    t0 = time.perf_counter()
    for g, info in zip(gates, infos):
        oracle.apply_gate(dims, psi, g)
        done += 1
        updates += info["updated"]
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {len(gates)} gates on the full D={math.prod(dims)} state "
                      f"(FP64 oracle, one thread, {dt:.1f} s)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--gates", type=int, default=500)
    ap.add_argument("--no-c64", action="store_true", help="skip the complex64 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--small", action="store_true", help="2^10 x 3^6 x 4^2 register (quick check)")
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

    res = {"c128": run_precision(qd, dims, gates, "c128", upload, args.steps, args.warmup)}
    if not args.no_c64:
        res["c64"] = run_precision(qd, dims, gates, "c64", upload, args.steps, args.warmup)
    cpu = None
    if host is not None:
        infos = [qd.gate_info(dims, g.targets, g.U, g.controls, g.values, "c128") for g in gates]
        cpu = cpu_baseline(dims, gates, host, infos, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.3e} updates/s ({cpu['sample']})")

    h = res["c128"]
    workload = (f"large: dims {'2^10 x 3^6 x 4^2' if args.small else '2^14 x 3^8 x 4^2'} (D={D}), complex128, "
                f"{len(gates)}-gate circuit (seed {circuits.SEEDS['large']}), Gaussian initial state in HBM")
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
        "config": {"workload": workload, "D": D, "gates": len(gates), "precision": "c128"},
        "algorithmic_GBps": h["algorithmic_GBps"],
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "kernels": h["kernels"],
        "norm_last_step": h["norm_last_step"],
    }
    if "c64" in res:
        c = res["c64"]
        line["c64"] = {"value": c["value"], "unit": "updates/s", "dtype": "f32", "ms_per_step": c["ms_per_step"],
                       "algorithmic_GBps": c["algorithmic_GBps"], "roofline": c["roofline"],
                       "norm_last_step": c["norm_last_step"], "kernels": c["kernels"]}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
