"""Benchmark of the IBLB wetting step on one MI355X.

A step is one full time step of the hot path (nodal forces, spreading,
fused stream-collide, interpolation and advection) over the spreading
workload: a 128x128x64 box (1,048,576 cells) with one 10,242-node droplet
relaxing from a 150 degree cap toward 60 degrees, FP32 storage, each step
replayed as a hipGraph.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + IB nodes/s, % HBM roofline; FP16-storage & batched vs FP32 at stated error"
HBM_PEAK_GBS = 8000.0
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3}
ELEM = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}


def algorithmic_bytes_per_step(wl, storage: str, band_cells: int) -> float:
    """Populations read once and written once (2 x 19 x element size per
    cell) plus, in the tiles near the mesh, the spread force read and the
    velocity written (2 x 3 x compute size)."""
    real = 8 if storage == "f64" else 4
    return wl.cells * 2 * 19 * ELEM[storage] + band_cells * 2 * 3 * real


def band_cells_of(sim, wl) -> int:
    """Cells of the stamped 4x4x4 tiles at the current positions."""
    total = 0
    for b in range(len(wl.boxes)):
        _, flags = sim.compute_spread(b)
        total += int(flags.sum()) * 64
    return total


def cpu_baseline(wl, seconds: float):
    import oracle
    sim = oracle.OracleSim(wl)
    sim.step(1)  # first-touch of the arrays outside the timing
    t0 = time.perf_counter()
    n = 0
    while True:
        sim.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= 10000:
            break
    return {"value": wl.cells * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} steps of the {wl.name} workload after its first step "
                      f"({dt:.1f} s, FP64, OpenMP over z-slabs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_17463_amd as P
    from iblb_inputs import configs

    wl = configs.spreading_c2()
    flags = P.IBLB_FLAG_GRAPH | (0 if args.no_autotune else P.IBLB_FLAG_AUTOTUNE)
    dev_scale = 4096.0 if args.storage == "f16dev" else 1.0
    sim = P.Simulation(wl, storage=STORAGE[args.storage], flags=flags, dev_scale=dev_scale)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    drops, boxes = sim.observables()

    cells, nodes = wl.cells, wl.nodes
    mlups = cells * args.steps / dt / 1e6
    # dominant kernel: fused stream-collide, timed alone with HIP events on
    # the library's stream, same launch shape as in the timed steps
    band = band_cells_of(sim, wl)
    k1_ms = sim.time_stream_collide(reps=200)
    bytes_k1 = algorithmic_bytes_per_step(wl, args.storage, band)
    achieved = bytes_k1 / (k1_ms * 1e-3) / 1e9
    launch = sim.get_launch()
    out = {
        "metric": METRIC, "value": round(mlups, 3), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "cells": cells, "ib_nodes": nodes,
                   "storage": args.storage, "graph": True, "k1_launch": list(launch)},
        "ib_nodes_per_s": nodes * args.steps / dt,
        "step_roofline_frac": (bytes_k1 + nodes * 150.0) * args.steps / dt / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_stream_collide", "kernel_ms": k1_ms,
                     "bytes_per_launch": bytes_k1, "band_cells": band},
        "observables": {"height": drops[0]["height"], "contact_radius": drops[0]["contact_radius"],
                        "volume": drops[0]["volume"], "mass": boxes[0]["mass"]},
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(configs.spreading_c2(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
