"""Benchmark of the IBLB wetting step on one MI355X.

A step is one full time step of the hot path (triangle and node forces,
spreading, fused stream-collide, interpolation and advection), replayed as
hipGraphs.  The headline workload is the spreading run: a 128x128x64 box
(1,048,576 cells) with one 10,242-node droplet relaxing from a 150 degree
cap toward 60 degrees, FP32 population storage.  One JSON line is printed;
besides the headline it carries:
  - the observable error of the FP32 run against the stored FP64 oracle
    trace of the same run (tests/golden/spreading_trace_oracle.json);
  - the same run with FP16- and BF16-deviation storage (speed and error);
  - the bulk stream-collide kernel on an HBM-resident 256x256x128 box;
  - the 64-box batched workload in one context against 64 sequential runs;
  - the FP64 oracle timed on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from dataclasses import replace

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + IB nodes/s, % HBM roofline; FP16-storage & batched vs FP32 at stated error"
HBM_PEAK_GBS = 8000.0
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3}
ELEM = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}
BYTES_PER_NODE = 150.0  # per IB node and step: q, phi, weights, CSR, triangle records
TRACE = os.path.join(ROOT, "tests", "golden", "spreading_trace_oracle.json")
TRAFFIC = os.path.join(ROOT, "profiles", "bulk_collide_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("iblb_device.h", "iblb_fluid.hip", "iblb_internal.h"):
        with open(os.path.join(ROOT, "paper_2604_17463_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cell_bytes(storage: str) -> int:
    """Algorithmic bytes per cell update: every population read once and
    written once."""
    return 2 * 19 * ELEM[storage]


def make_sim(wl, storage, autotune=True):
    import paper_2604_17463_amd as P
    flags = P.IBLB_FLAG_GRAPH | (P.IBLB_FLAG_AUTOTUNE if autotune else 0)
    return P.Simulation(wl, storage=STORAGE[storage], flags=flags,
                        dev_scale=4096.0 if storage == "f16dev" else 1.0)


def timed_steps(sim, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def oracle_errors(drop, box, step):
    """Relative error of the GPU observables against the stored oracle trace
    at the same step (None when the trace is absent or does not reach it)."""
    if not os.path.exists(TRACE):
        return None
    with open(TRACE) as fh:
        tr = json.load(fh)
    rows = {r["step"]: r for r in tr["rows"]}
    if step not in rows:
        return None
    r = rows[step]
    out = {"step": step}
    for k in ("height", "contact_radius", "volume", "area"):
        out[k] = abs(drop[k] - r[k]) / abs(r[k])
    out["mass"] = abs(box["mass"] - r["mass"]) / r["mass"]
    return out


def traffic_record():
    """HBM bytes per bulk launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec


def cpu_baseline(wl, seconds: float):
    import oracle
    sim = oracle.OracleSim(wl)
    sim.step(1)  # first touch of the arrays outside the timing
    t0 = time.perf_counter()
    n = 0
    while True:
        sim.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= 10000:
            break
    return {"value": round(wl.cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} steps of the {wl.name} workload after its first step "
                      f"({dt:.1f} s, FP64, OpenMP over z-slabs)"}


def run_spreading(storage, warmup, steps, autotune=True):
    from iblb_inputs import configs
    wl = configs.spreading_c2()
    sim = make_sim(wl, storage, autotune)
    sim.step(warmup)
    dt = timed_steps(sim, steps)
    drops, boxes = sim.observables()
    return wl, sim, dt, drops[0], boxes[0]


def variants(args, f32_drop, total_steps):
    from iblb_inputs import configs
    from iblb_inputs.configs import Box, Workload
    out = {}
    # reduced-precision population storage on the same spreading run
    for st in ("f16dev", "bf16dev"):
        wl, sim, dt, d, b = run_spreading(st, args.warmup, args.steps)
        k1 = sim.time_stream_collide(reps=100)
        out[st] = {"mlups": round(wl.cells * args.steps / dt / 1e6, 3),
                   "ms_per_step": dt / args.steps * 1e3,
                   "bulk_kernel_ms": k1,
                   "bulk_GBs": round(wl.cells * cell_bytes(st) / (k1 * 1e-3) / 1e9, 1),
                   "rel_err_vs_f32": {k: abs(d[k] - f32_drop[k]) / abs(f32_drop[k])
                                      for k in ("height", "contact_radius", "volume")},
                   "rel_err_vs_oracle": oracle_errors(d, b, total_steps)}
        sim.close()
    # HBM-resident box (1.3 GB of FP32 populations, beyond the 256 MB cache)
    big = Workload("box-256x256x128", [Box(256, 256, 128, tau=0.6)], [])
    for st in ("f32", "f16dev"):
        sim = make_sim(big, st)
        sim.time_stream_collide(reps=5)
        k1 = sim.time_stream_collide(reps=50)
        gbs = big.cells * cell_bytes(st) / (k1 * 1e-3) / 1e9
        out[f"hbm_box_{st}"] = {"workload": big.name, "bulk_kernel_ms": k1,
                                "mlups": round(big.cells / (k1 * 1e-3) / 1e6, 1),
                                "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                "launch": list(sim.get_launch())}
        sim.close()
    # batched: 64 uneven boxes in one context vs 64 sequential contexts
    if not args.no_batched:
        wl = configs.batched_c4()
        nb_steps = args.batched_steps
        sim = make_sim(wl, "f32")
        sim.step(20)
        dt = timed_steps(sim, nb_steps)
        sim.close()
        seq_time = 0.0
        for k in range(len(wl.boxes)):
            one = Workload("one", [wl.boxes[k]], [replace(wl.droplets[k], box=0)], storage=1)
            s = make_sim(one, "f32")
            s.step(20)
            seq_time += timed_steps(s, nb_steps)
            s.close()
        out["batched"] = {"workload": wl.name, "boxes": len(wl.boxes), "cells": wl.cells,
                          "ib_nodes": wl.nodes, "steps": nb_steps,
                          "mlups": round(wl.cells * nb_steps / dt / 1e6, 3),
                          "ib_nodes_per_s": wl.nodes * nb_steps / dt,
                          "sequential_mlups": round(wl.cells * nb_steps / seq_time / 1e6, 3),
                          "speedup_vs_sequential": seq_time / dt}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    wl, sim, dt, drop, box = run_spreading(args.storage, args.warmup, args.steps,
                                           not args.no_autotune)
    cells, nodes = wl.cells, wl.nodes
    mlups = cells * args.steps / dt / 1e6
    # dominant kernel: the bulk stream-collide, timed alone with HIP events
    # on the library's stream in the launch shape the timed steps used
    _, flags = sim.compute_spread(0)
    band = int(flags.sum()) * 64
    k1_ms = sim.time_stream_collide(reps=200)
    bytes_k1 = cells * cell_bytes(args.storage)
    achieved = bytes_k1 / (k1_ms * 1e-3) / 1e9
    launch = sim.get_launch()
    sim.close()
    tr = traffic_record()
    traffic = None
    if (tr and tr.get("workload") == wl.name and tr.get("storage") == args.storage
            and tuple(tr.get("launch", ())) == tuple(launch)):
        traffic = tr["hbm_bytes_per_launch"]
    out = {
        "metric": METRIC, "value": round(mlups, 3), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "cells": cells, "ib_nodes": nodes,
                   "storage": args.storage, "graph": True, "bulk_launch": list(launch)},
        "ib_nodes_per_s": nodes * args.steps / dt,
        "bytes_per_cell_update": cell_bytes(args.storage),
        "step_roofline_frac": (bytes_k1 + nodes * BYTES_PER_NODE) * args.steps / dt
        / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_bulk (fused pull-stream/collide, every cell)",
                     "kernel_ms": k1_ms, "bytes_per_launch": bytes_k1, "band_cells": band},
        "observables": {"step": drop["step"], "height": drop["height"],
                        "contact_radius": drop["contact_radius"], "volume": drop["volume"],
                        "mass": box["mass"]},
        "rel_err_vs_oracle": oracle_errors(drop, box, args.warmup + args.steps),
    }
    if not args.no_variants:
        out["variants"] = variants(args, drop, args.warmup + args.steps)
    if not args.no_cpu_baseline:
        from iblb_inputs import configs
        out["cpu_baseline"] = cpu_baseline(configs.spreading_c2(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
