"""Driver for rocprofv3 runs of the IBLB kernels.

    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_2604_17463_amd.profiling [--bulk ...]
    rocprofv3 --pmc WRITE_SIZE -d OUT -- python -m paper_2604_17463_amd.profiling [--bulk ...]
    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2604_17463_amd.profiling [--bulk ...]

By default (or with --bulk NAME=LAUNCH ...) a plain device copy of a known
size (torch's copy kernel) first serves as the calibration of the memory
counters; then the bulk stream-collide kernel runs over every cell, 3 +
`reps` times, on each named workload (spreading, box256, multidroplet,
batched) in the given launch shape (threads_x, rows, rows_per_thread,
streaming_stores, max_workgroups).

With --steps WORKLOAD N it instead runs N graph-replayed FP32 steps of a
named workload after 20 warm-up steps and prints the step time and the
band cells of the last step, for kernel traces and counters of whole steps.
With --launch the bulk launch and step schedule are set as given and
nothing is autotuned, so that a trace holds only the steps' own launches;
without it the context autotunes at init (its candidate launches then
appear in a trace too).  --eager launches the kernels one by one instead of
replaying graphs.

With --copy GIB it instead copies a device buffer of that size (torch's copy
kernel) 3 + `reps` times, the plain-copy ceiling of the memory system at
that footprint.
"""
from __future__ import annotations

import argparse
import json


WORKLOADS = ("spreading", "box256", "multidroplet", "batched")


def _workload(name):
    from iblb_inputs import configs
    from iblb_inputs.configs import Box, Workload
    if name == "box256":
        return Workload("box-256x256x128", [Box(256, 256, 128, tau=0.6)], [])
    return {"spreading": configs.spreading_c2, "batched": configs.batched_c4,
            "multidroplet": configs.multidroplet_c5}[name]()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--storage", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--bulk", nargs="+", default=["spreading=128,1,1,0,1024", "box256=256,1,1,1,0"],
                    metavar="NAME=LAUNCH",
                    help="workloads and bulk launches (threads_x,rows,rows_per_thread,"
                         "streaming_stores,max_workgroups) for the counter runs")
    ap.add_argument("--steps", nargs=2, metavar=("WORKLOAD", "N"),
                    help="run N steps of spreading, batched or multidroplet instead")
    ap.add_argument("--launch", type=int, nargs=6, default=None,
                    help="with --steps: bulk launch and schedule to set (no autotuning)")
    ap.add_argument("--eager", action="store_true", help="with --steps: no graph replay")
    ap.add_argument("--copy", type=float, default=0.0, metavar="GIB",
                    help="time a device copy of this many GiB instead")
    args = ap.parse_args()
    import torch
    if args.steps:
        return run_steps(args.steps[0], int(args.steps[1]), args.launch, args.eager)
    if args.copy > 0:
        return run_copy(args.copy, args.reps)

    import paper_2604_17463_amd as P

    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    res = {"copy_bytes_each_way": n * 4}
    for item in args.bulk:
        name, launch = item.split("=")
        launch = [int(v) for v in launch.split(",")]
        assert name in WORKLOADS, name
        wl = _workload(name)
        sim = P.Simulation(wl, storage=args.storage, dev_scale=4096.0 if args.storage == 2 else 1.0)
        sim.set_launch(*launch)
        sim.time_stream_collide(reps=3)
        ms = sim.time_stream_collide(reps=args.reps)
        # keyed by the whole NAME=LAUNCH item: one workload may be timed in
        # several launch shapes
        res[item] = {"workload": wl.name, "cells": wl.cells, "bulk_ms": ms,
                     "launch": list(sim.get_launch())}
        sim.close()
        print(json.dumps({item: res[item]}), flush=True)
    print(json.dumps(res), flush=True)


def run_copy(gib, reps):
    """Device-to-device copy of `gib` GiB (torch's copy kernel): mean time
    and rate over `reps` copies after 3 untimed ones."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_each_way": n * 4, "ms": ms,
                      "GBs_read_plus_write": 2 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)


def run_steps(name, n, launch=None, eager=False):
    import time

    import numpy as np
    import torch

    import paper_2604_17463_amd as P
    wl = _workload(name)
    flags = (0 if eager else P.IBLB_FLAG_GRAPH) | (0 if launch else P.IBLB_FLAG_AUTOTUNE)
    sim = P.Simulation(wl, storage=P.IBLB_F32, flags=flags)
    if launch:
        sim.set_launch(*launch)
    sim.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    band = 0
    tx, ty, tz = P.band_tile()
    for b, box in enumerate(wl.boxes):
        _, flags_b = sim.compute_spread(b, want_F=False)
        # cells of the stamped tiles that lie in the box (edge tiles are partial)
        cz = np.minimum(tz, box.nz - tz * np.arange(flags_b.shape[0]))
        cy = np.minimum(ty, box.ny - ty * np.arange(flags_b.shape[1]))
        cx = np.minimum(tx, box.nx - tx * np.arange(flags_b.shape[2]))
        band += int((flags_b * cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).sum())
    print(json.dumps({"workload": wl.name, "cells": wl.cells, "steps": n, "ms_per_step": dt / n * 1e3,
                      "launch": list(sim.get_launch()), "graph": not eager,
                      "band_cells_at_end": band}), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
