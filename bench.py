"""Benchmark of the IBLB wetting step on one MI355X.

A step is one full time step of the hot path (triangle and node forces,
spreading, fused stream-collide, interpolation and advection), replayed as
hipGraphs.  The headline workload is the largest single-GPU configuration:
a 512x512x256 box (67,108,864 cells, 10.2 GB of FP32 populations per
buffer pair) with 16 droplets of 10,242 nodes each on a 4x4 grid over the
wetting wall, FP32 population storage.  One JSON line is printed; besides
the headline it carries:
  - the roofline of the dominant kernel (the fused stream-collide over every
    cell, timed with HIP events on the library's stream in the step's launch
    shape) and the step-level fraction of HBM peak;
  - the same box with FP16-deviation storage against FP32 over the
    configured 5,000 steps (speed-up, worst observable error);
  - the 128x128x64 spreading run (cache-resident: its two population
    buffers fit in the 256 MB last-level cache) in FP32, FP16- and
    BF16-deviation storage, with observable errors against the stored FP64
    oracle trace (tests/golden/spreading_trace_oracle.json);
  - the bulk stream-collide kernel alone on an HBM-resident 256x256x128 box;
  - the 256x256x128 precision workload (40,962-node droplet, tau 0.6 and
    1.0) in FP64, FP32, FP16- and BF16-deviation storage over its configured
    10,000 steps, with observable errors against the stored FP64 oracle trace
    and against the FP64 run;
  - the 64-box batched workload in one context, FP32 and FP16-deviation,
    against 64 sequential FP32 contexts;
  - the FP64 oracle timed on the host cores on the headline workload
    (cpu_baseline);
  - opt-in: the paper's own spreading runs at their scale (--paper-spreading),
    the two wetting runs of Sec. 4 (--paper-sec4), and the free droplet in
    shear at the paper's parameters (--paper-shear).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
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
BYTES_PER_BAND_CELL = 24.0  # per cell of a stamped tile: spread force read, velocity write
TRACE = os.path.join(ROOT, "tests", "golden", "spreading_trace_oracle.json")
PTRACE = os.path.join(ROOT, "tests", "golden", "precision_trace_oracle_tau{tau:g}.json")
MTRACE = os.path.join(ROOT, "tests", "golden", "multidroplet_trace_oracle.json")
OBS = ("height", "contact_radius", "volume", "area")
TRAFFIC = os.path.join(ROOT, "profiles", "bulk_collide_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("iblb_device.h", "iblb_fluid.hip", "iblb_internal.h", "iblb_api.hip"):
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


def rel_errors(got, ref, keys=OBS):
    return {k: abs(got[k] - ref[k]) / abs(ref[k]) for k in keys}


def bulk_rate(sim, cells, storage, reps=50):
    """Bulk kernel alone over every cell, in the context's launch shape:
    (ms, GB/s of algorithmic traffic)."""
    sim.time_stream_collide(reps=3)
    ms = sim.time_stream_collide(reps=reps)
    return ms, cells * cell_bytes(storage) / (ms * 1e-3) / 1e9


def timed_steps(sim, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def band_cells(sim, b=0):
    """Cells of the band tiles the node pass stamps at the current state
    (edge tiles counted with their cells inside the box)."""
    import numpy as np

    import paper_2604_17463_amd as P
    box = sim.wl.boxes[b]
    tx, ty, tz = P.band_tile()
    _, flags = sim.compute_spread(b, want_F=False)
    cz = np.minimum(tz, box.nz - tz * np.arange(flags.shape[0]))
    cy = np.minimum(ty, box.ny - ty * np.arange(flags.shape[1]))
    cx = np.minimum(tx, box.nx - tx * np.arange(flags.shape[2]))
    return int((flags * cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).sum())


def oracle_errors(sim):
    """Advance the spreading run to the next row of the stored oracle trace
    (rows every 100 steps) and return the relative error of the observables
    there, with the step used; None when the trace is absent or ends
    earlier."""
    if not os.path.exists(TRACE):
        return None
    with open(TRACE) as fh:
        tr = json.load(fh)
    rows = {r["step"]: r for r in tr["rows"]}
    d, _ = sim.observables()
    now = d[0]["step"]
    target = min((s for s in rows if s >= now), default=None)
    if target is None:
        return None
    if target > now:
        sim.step(target - now)
    d, b = sim.observables()
    r = rows[target]
    out = {"step": target}
    for k in ("height", "contact_radius", "volume", "area"):
        out[k] = abs(d[0][k] - r[k]) / abs(r[k])
    out["mass"] = abs(b[0]["mass"] - r["mass"]) / r["mass"]
    return out


def headline_oracle_errors(sim, wl):
    """Advance the headline run to the next row of the stored oracle trace of
    its box (rows every 25 steps) and return, per observable, the largest
    relative error over its droplets there (mass: of the box), with the step
    used; None when the trace is absent, of another workload, or ends
    earlier."""
    if not os.path.exists(MTRACE):
        return None
    from iblb_inputs.configs import workload_hash
    with open(MTRACE) as fh:
        tr = json.load(fh)
    if tr.get("workload_sha256") != workload_hash(wl):
        return None
    rows = {r["step"]: r for r in tr["rows"]}
    d, _ = sim.observables()
    now = d[0]["step"]
    target = min((s for s in rows if s >= now), default=None)
    if target is None:
        return None
    if target > now:
        sim.step(target - now)
    d, b = sim.observables()
    r = rows[target]
    out = {"step": target}
    for k in ("height", "contact_radius", "volume", "area"):
        out[k] = max(abs(g[k] - o[k]) / abs(o[k]) for g, o in zip(d, r["droplets"]))
    out["mass"] = abs(b[0]["mass"] - r["mass"]) / r["mass"]
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


def counted_traffic(rec, workload: str, storage: str, launch):
    """HBM bytes per bulk launch counted for this workload and storage in
    this launch shape (threads_x, rows, rows per thread, streaming stores,
    grid cap), from the record's entry for that shape, or None."""
    if not rec or rec.get("workload") != workload or rec.get("storage") != storage:
        return None
    for e in [rec] + list(rec.get("launches", [])):
        if tuple(e.get("launch", ()))[:5] == tuple(launch)[:5]:
            return e["hbm_bytes_per_launch"]
    return None


def cpu_baseline(wl, seconds: float):
    """The oracle on the host cores (all the process may use, then one
    thread), on the same workload from its initial state: steps until
    `seconds` have passed, then one step on one thread."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    oracle.set_threads(cores)
    sim = oracle.OracleSim(wl)
    sim.step(1)  # first touch of the arrays outside the timing
    t0 = time.perf_counter()
    n = 0
    while True:
        sim.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    used = oracle.num_threads()
    oracle.set_threads(1)
    t1 = time.perf_counter()
    sim.step(1)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": round(wl.cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": used,
            "kind": "oracle", "value_1_thread": round(wl.cells / dt1 / 1e6, 3),
            "sample": f"{n} steps of the {wl.name} workload ({wl.cells:,} cells, {wl.nodes:,} IB "
                      f"nodes) after its first step ({dt:.1f} s, FP64, OpenMP over z-slabs on "
                      f"{used} threads); one thread: 1 step in {dt1:.1f} s"}


def spreading_variants(args):
    """The 128x128x64 spreading run (cache-resident) in three storages."""
    from iblb_inputs import configs
    out = {}
    f32 = None
    for st in ("f32", "f16dev", "bf16dev"):
        wl = configs.spreading_c2()
        sim = make_sim(wl, st)
        sim.step(args.spreading_warmup)
        dt = timed_steps(sim, args.spreading_steps)
        d, _ = sim.observables()
        k1, gbs = bulk_rate(sim, wl.cells, st, reps=100)
        r = {"workload": wl.name, "cache_resident": True,
             "mlups": round(wl.cells * args.spreading_steps / dt / 1e6, 3),
             "ib_nodes_per_s": wl.nodes * args.spreading_steps / dt,
             "ms_per_step": dt / args.spreading_steps * 1e3,
             "bulk_kernel_ms": k1, "bulk_GBs_cache_resident": round(gbs, 1),
             "launch": list(sim.get_launch())}
        if st == "f32":
            r["mesh_kernels_ms"] = sim.time_mesh_chain(reps=100)
            f32 = d[0]
        else:
            r["rel_err_vs_f32"] = {k: abs(d[0][k] - f32[k]) / abs(f32[k])
                                   for k in ("height", "contact_radius", "volume")}
            r["speedup_vs_f32"] = out["f32"]["ms_per_step"] / r["ms_per_step"]
        r["rel_err_vs_oracle"] = oracle_errors(sim)
        sim.close()
        out[st] = r
    return out


def hbm_box():
    from iblb_inputs.configs import Box, Workload
    big = Workload("box-256x256x128", [Box(256, 256, 128, tau=0.6)], [])
    out = {}
    for st in ("f32", "f16dev"):
        sim = make_sim(big, st)
        k1, gbs = bulk_rate(sim, big.cells, st)
        out[st] = {"workload": big.name, "bulk_kernel_ms": k1,
                   "mlups": round(big.cells / (k1 * 1e-3) / 1e6, 1),
                   "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                   "launch": list(sim.get_launch())}
        sim.close()
    return out


def precision(args):
    """FP64 / FP32 / FP16 / BF16 storage on the precision workload over its
    configured length, against the stored oracle trace and the FP64 run."""
    from iblb_inputs import configs
    out = {}
    for tau in (0.6, 1.0):
        wl = configs.precision_c3(tau=tau, steps=args.precision_steps)
        ref_path = PTRACE.format(tau=tau)
        oracle_row = None
        if os.path.exists(ref_path):
            with open(ref_path) as fh:
                tr = json.load(fh)
            oracle_row = {r["step"]: r for r in tr["rows"]}.get(args.precision_steps)
        runs = {}
        for st in ("f64", "f32", "f16dev", "bf16dev"):
            sim = make_sim(wl, st)
            sim.step(20)
            dt = timed_steps(sim, args.precision_steps - 20)
            d, b = sim.observables()
            ms, gbs = bulk_rate(sim, wl.cells, st)
            obs = {k: d[0][k] for k in OBS}
            obs["mass"] = b[0]["mass"]
            runs[st] = {"mlups": round(wl.cells * (args.precision_steps - 20) / dt / 1e6, 1),
                        "ms_per_step": dt / (args.precision_steps - 20) * 1e3,
                        "bulk_GBs": round(gbs, 1), "bulk_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "launch": list(sim.get_launch()), "obs": obs}
            sim.close()
        for st, r in runs.items():
            r["rel_err_vs_f64_gpu"] = rel_errors(r["obs"], runs["f64"]["obs"], OBS + ("mass",))
            if oracle_row is not None:
                r["rel_err_vs_oracle"] = rel_errors(r["obs"], oracle_row, OBS + ("mass",))
            r["speedup_vs_f32"] = runs["f32"]["ms_per_step"] / r["ms_per_step"]
        out[f"tau{tau:g}"] = {"workload": wl.name, "steps": args.precision_steps,
                              "oracle_trace": oracle_row is not None, "runs": runs}
    return out


def large_precision(args):
    """The headline box in FP32 and FP16-deviation storage over the configured
    length; the worst relative difference of each droplet observable,
    sampled every `every` steps."""
    from iblb_inputs import configs
    wl = configs.multidroplet_c5()
    n, every = args.large_steps, max(1, args.large_steps // 10)
    runs, trace = {}, {}
    for st in ("f32", "f16dev"):
        sim = make_sim(wl, st)
        sim.step(20)
        dt, rows = 0.0, []
        done = 0
        while done < n:
            k = min(every, n - done)
            dt += timed_steps(sim, k)
            done += k
            drops, boxes = sim.observables()
            rows.append(([{key: d[key] for key in OBS} for d in drops], boxes[0]["mass"]))
        ms, gbs = bulk_rate(sim, wl.cells, st, reps=20)
        runs[st] = {"mlups": round(wl.cells * n / dt / 1e6, 1), "ib_nodes_per_s": wl.nodes * n / dt,
                    "ms_per_step": dt / n * 1e3, "bulk_GBs": round(gbs, 1),
                    "bulk_frac": round(gbs / HBM_PEAK_GBS, 4), "launch": list(sim.get_launch())}
        trace[st] = rows
        sim.close()
    worst = {k: max(abs(a[k] - b[k]) / abs(b[k])
                    for (da, _), (db, _) in zip(trace["f16dev"], trace["f32"]) for a, b in zip(da, db))
             for k in OBS}
    worst["mass"] = max(abs(ma - mb) / mb for (_, ma), (_, mb) in zip(trace["f16dev"], trace["f32"]))
    return {"workload": wl.name, "cells": wl.cells, "ib_nodes": wl.nodes, "steps": n + 20,
            "compared_every": every, "runs": runs, "f16dev_worst_rel_err_vs_f32": worst,
            "f16dev_speedup_vs_f32": runs["f32"]["ms_per_step"] / runs["f16dev"]["ms_per_step"]}


def batched(args):
    """64 uneven boxes in one context (FP32 and FP16-deviation) against 64
    sequential FP32 contexts; the FP16 run's worst observable error against
    the FP32 batch."""
    from iblb_inputs import configs
    from iblb_inputs.configs import Workload
    wl = configs.batched_c4()
    nb_steps = args.batched_steps
    res, obs = {}, {}
    for st in ("f32", "f16dev"):
        sim = make_sim(wl, st)
        sim.step(20)
        dt = timed_steps(sim, nb_steps)
        drops, boxes = sim.observables()
        obs[st] = ([{k: d[k] for k in OBS} for d in drops], [b["mass"] for b in boxes])
        res[st] = {"mlups": round(wl.cells * nb_steps / dt / 1e6, 3),
                   "ib_nodes_per_s": wl.nodes * nb_steps / dt, "ms_per_step": dt / nb_steps * 1e3,
                   "launch": list(sim.get_launch())}
        sim.close()
    seq_time = 0.0
    for k in range(len(wl.boxes)):
        one = Workload("one", [wl.boxes[k]], [replace(wl.droplets[k], box=0)], storage=1)
        s = make_sim(one, "f32")
        s.step(20)
        seq_time += timed_steps(s, nb_steps)
        s.close()
    worst = {k: max(abs(a[k] - b[k]) / abs(b[k]) for a, b in zip(obs["f16dev"][0], obs["f32"][0]))
             for k in OBS}
    worst["mass"] = max(abs(a - b) / b for a, b in zip(obs["f16dev"][1], obs["f32"][1]))
    return {"workload": wl.name, "boxes": len(wl.boxes), "cells": wl.cells, "ib_nodes": wl.nodes,
            "steps": nb_steps, "runs": res,
            "sequential_f32_mlups": round(wl.cells * nb_steps / seq_time / 1e6, 3),
            "speedup_vs_sequential": seq_time / nb_steps * 1e3 / res["f32"]["ms_per_step"],
            "f16dev_worst_rel_err_vs_f32": worst,
            "f16dev_speedup_vs_f32": res["f32"]["ms_per_step"] / res["f16dev"]["ms_per_step"]}


def paper_spreading(taus, n_tmu):
    """The paper's own spreading runs (Sec. 3) at their scale: 250x250x150,
    118,580-triangle mesh, R0 = 60, 90 -> 60 deg, for each tau over n_tmu
    units t_mu = mu R0 / sigma; h / R0 every t_mu / 2."""
    from iblb_inputs import configs
    out = {}
    for tau in taus:
        wl = configs.paper_spreading(tau)
        sim = make_sim(wl, "f32")
        tmu, r0 = wl.extra["t_mu"], wl.extra["r0"]
        every = max(1, int(round(tmu / 2)))
        n = int(round(2 * n_tmu))
        rows, dt = [], 0.0
        for i in range(1, n + 1):
            dt += timed_steps(sim, every)
            d, _ = sim.observables()
            rows.append([round(d[0]["step"] / tmu, 3), round(d[0]["height"] / r0, 5),
                         round(math.degrees(d[0]["theta_app"]), 3)])
            if i % 20 == 0:
                print(f"paper spreading tau {tau}: t/t_mu {rows[-1][0]:.1f} h/R0 {rows[-1][1]:.4f}",
                      file=sys.stderr, flush=True)
        sim.close()
        out[f"tau{tau:g}"] = {"workload": wl.name, "re": wl.extra["re"], "t_mu": tmu,
                              "steps": every * n, "mlups": round(wl.cells * every * n / dt / 1e6, 1),
                              "ib_nodes": wl.nodes, "t_over_tmu_h_over_r0_theta": rows}
        print(f"paper spreading tau {tau}: h/R0 {rows[-1][1]:.4f} at t/t_mu {rows[-1][0]:.1f}",
              file=sys.stderr, flush=True)
    return out


def half_profile(q, tris, cx, cy, levels=12):
    """Half-profile of a droplet mesh: at `levels` heights evenly spaced
    between its lowest and highest node, the mean distance from the vertical
    axis through (cx, cy) of the points where mesh edges cross that plane."""
    import numpy as np
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    a, b = q[e[:, 0]], q[e[:, 1]]
    z0, z1 = q[:, 2].min(), q[:, 2].max()
    out = []
    for k in range(levels):
        z = z0 + (k + 0.5) / levels * (z1 - z0)
        m = (a[:, 2] - z) * (b[:, 2] - z) < 0
        s = (z - a[m, 2]) / (b[m, 2] - a[m, 2])
        p = a[m] + s[:, None] * (b[m] - a[m])
        out.append((z, float(np.hypot(p[:, 0] - cx, p[:, 1] - cy).mean())))
    return out


def paper_sec4(n_cap, n_neck):
    """The two wetting runs of the paper's Sec. 4 at their scale: the 90 deg
    cap spreading to 45 deg (tau = 0.59, 250x250x150) over n_cap t_mu, and
    the sphere released at xi above the wall (tau = 0.56, 300x300x250) over
    n_neck t_mu; h / R0, r_c / R0 and the apparent angle every t_mu / 2, and
    half-profiles (z / R0, r / R0) at the times the paper shows."""
    from iblb_inputs import configs
    out = {}
    for key, wl, n_tmu, shown in (("cap45", configs.paper_cap45(), n_cap, (0, 4, 10, 70)),
                                  ("neck", configs.paper_neck(), n_neck, (3, 18, 30, 48))):
        sim = make_sim(wl, "f32")
        tmu, r0 = wl.extra["t_mu"], wl.extra["r0"]
        tris = wl.droplets[0].tris
        every = max(1, int(round(tmu / 2)))
        n = int(round(2 * n_tmu))
        want = {int(round(2 * t)) for t in shown if t <= n_tmu}
        rows, profiles, dt = [], {}, 0.0
        d0 = sim.observables()[0][0]

        def profile(d):
            return [[round(z / r0, 4), round(r / r0, 4)]
                    for z, r in half_profile(sim.read_nodes(0), tris, d["cx"], d["cy"])]
        if 0 in want:
            profiles["0"] = profile(d0)
        for i in range(1, n + 1):
            dt += timed_steps(sim, every)
            d = sim.observables()[0][0]
            rows.append([round(d["step"] / tmu, 3), round(d["height"] / r0, 5),
                         round(d["contact_radius"] / r0, 5), round(math.degrees(d["theta_app"]), 3)])
            if i in want:
                profiles[f"{i / 2:g}"] = profile(d)
            if i % 20 == 0:
                print(f"paper sec4 {key}: t/t_mu {rows[-1][0]:.1f} h/R0 {rows[-1][1]:.4f}",
                      file=sys.stderr, flush=True)
        sim.close()
        out[key] = {"workload": wl.name, "re": wl.extra["re"], "t_mu": tmu, "steps": every * n,
                    "mlups": round(wl.cells * every * n / dt / 1e6, 1), "ib_nodes": wl.nodes,
                    "volume_drift": d["volume"] / d0["volume"] - 1.0,
                    "t_over_tmu_h_rc_over_r0_theta": rows, "half_profiles_z_r_over_r0": profiles}
    return out


def paper_shear(n_cap):
    """Sec. 4's free droplet in shear at the paper's own parameters: R0 = 19,
    Re = 0.01, Ca = 0.05, tau_in = tau_out = 1 (lambda = 1), an ico5 mesh,
    walls 8 R0 from the centre (204 x 152 x 304).  The fluid starts as the
    Couette flow (its BGK equilibrium, built here from the library's velocity
    set).  D / D_inf every capillary time mu R0 / sigma over n_cap of them;
    the paper reports its IBLB run 2.7 % from D_inf."""
    import numpy as np

    import paper_2604_17463_amd as P
    from iblb_inputs import configs
    wl = configs.shear_droplet(lam=1.0, r=19.0, shape=(204, 152, 304), level=5)
    box, gamma = wl.boxes[0], wl.extra["shear_rate"]
    sim = make_sim(wl, "f32")
    c, w = P.velocity_set()
    u = gamma * (np.arange(box.nz) + 0.5 - box.nz / 2.0)
    cu = c[:, 0][:, None] * u[None, :]
    feq = w[:, None] * box.rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u[None, :] ** 2)
    sim.write_state(np.ascontiguousarray(
        np.broadcast_to(feq[:, :, None, None], (19, box.nz, box.ny, box.nx))))
    dinf = (19.0 + 16.0) / 32.0 * wl.extra["ca"]
    tcap = wl.extra["t_cap"]
    d0 = sim.observables()[0][0]
    rows, dt = [], 0.0
    for k in range(1, int(n_cap) + 1):
        dt += timed_steps(sim, int(round(k * tcap)) - int(round((k - 1) * tcap)))
        d = sim.observables()[0][0]
        rows.append([k, round(d["deformation"] / dinf, 5), round(math.degrees(d["inclination"]), 3)])
        print(f"paper shear: t/t_cap {k} D/D_inf {rows[-1][1]:.4f}", file=sys.stderr, flush=True)
    sim.close()
    return {"workload": wl.name, "cells": wl.cells, "ib_nodes": wl.nodes, "t_cap": tcap,
            "steps": int(round(n_cap * tcap)), "mlups": round(wl.cells * n_cap * tcap / dt / 1e6, 1),
            "d_inf": dinf, "final_rel_distance_from_d_inf": rows[-1][1] - 1.0,
            "paper_rel_distance": {"iblb": 0.027, "vof": 0.013},
            "volume_drift": d["volume"] / d0["volume"] - 1.0,
            "t_over_tcap_d_over_dinf_inclination_deg": rows}


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--spreading-steps", type=int, default=5000)
    ap.add_argument("--spreading-warmup", type=int, default=200)
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--precision-steps", type=int, default=10000)
    ap.add_argument("--large-steps", type=int, default=5000)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--paper-spreading", default="",
                    help="comma-separated tau values: also run the paper-scale spreading runs "
                         "(250x250x150, 118,580 triangles; about 2,500 steps/s)")
    ap.add_argument("--paper-tmu", type=float, default=50.0)
    ap.add_argument("--paper-sec4", action="store_true",
                    help="also run the two wetting runs of Sec. 4 at their scale (45 deg cap, "
                         "250x250x150; sphere released at the wall, 300x300x250)")
    ap.add_argument("--paper-sec4-tmu", type=float, nargs=2, default=(70.0, 50.0),
                    help="their lengths in t_mu")
    ap.add_argument("--paper-shear", type=float, default=0.0, metavar="N_CAP",
                    help="also run the free droplet in shear at the paper's R0 = 19 for N_CAP "
                         "capillary times (16 reach the plateau; about 10,800 steps each)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from iblb_inputs import configs
    wl = configs.multidroplet_c5()
    progress(f"headline {wl.name}: init and autotune")
    sim = make_sim(wl, args.storage, not args.no_autotune)
    sim.step(args.warmup)
    progress(f"headline: {args.steps} timed steps")
    dt = timed_steps(sim, args.steps)
    drops, boxes = sim.observables()
    cells, nodes = wl.cells, wl.nodes
    mlups = cells * args.steps / dt / 1e6
    # after the timed steps: the run advanced to the oracle trace's next row
    err_oracle = headline_oracle_errors(sim, wl) if args.storage == "f32" else None
    band = sum(band_cells(sim, b) for b in range(len(wl.boxes)))
    # dominant kernel: the bulk stream-collide over every cell, timed alone
    # with HIP events on the library's stream in the launch shape of the
    # timed steps
    k1_ms = sim.time_stream_collide(reps=3)
    k1_ms = sim.time_stream_collide(reps=50)
    # the mesh kernels alone (nodes/s over their time, without the fluid)
    mesh_ms = sim.time_mesh_chain(reps=20)
    bytes_k1 = cells * cell_bytes(args.storage)
    achieved = bytes_k1 / (k1_ms * 1e-3) / 1e9
    launch = sim.get_launch()
    sim.close()
    traffic = counted_traffic(traffic_record(), wl.name, args.storage, launch)
    step_bytes = bytes_k1 + band * BYTES_PER_BAND_CELL + nodes * BYTES_PER_NODE
    out = {
        "metric": METRIC, "value": round(mlups, 3), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "cells": cells, "ib_nodes": nodes, "droplets": len(wl.droplets),
                   "storage": args.storage, "graph": True, "launch": list(launch)},
        "ib_nodes_per_s": nodes * args.steps / dt,
        "ib_nodes_per_s_mesh_kernels": nodes / (mesh_ms * 1e-3),
        "mesh_kernels_ms": mesh_ms,
        "bytes_per_cell_update": cell_bytes(args.storage),
        "step_bytes": step_bytes,
        "step_roofline_frac": step_bytes * args.steps / dt / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_bulk (fused pull-stream/BGK-Guo collide over every cell; in the step it "
                               "skips the band tiles, which the band kernel computes beside it)",
                     "kernel_ms": k1_ms, "bytes_per_launch": bytes_k1, "band_cells": band,
                     "launch": list(launch)},
        "observables": {"step": drops[0]["step"], "mass": boxes[0]["mass"],
                        "height_mean": sum(d["height"] for d in drops) / len(drops),
                        "volume_total": sum(d["volume"] for d in drops)},
        "rel_err_vs_oracle": err_oracle,
        "parity": "tests/test_gpu_window.py: one step on windows of this box against the oracle",
    }
    if not args.no_variants:
        v = {}
        progress("spreading run (cache-resident) in three storages")
        v["spreading"] = spreading_variants(args)
        progress("bulk kernel on the HBM-resident 256x256x128 box")
        v["hbm_box"] = hbm_box()
        progress(f"precision workload, {args.precision_steps} steps in four storages")
        v["precision"] = precision(args)
        if not args.no_large:
            progress(f"headline box FP32 vs FP16, {args.large_steps} steps")
            v["large_fp16"] = large_precision(args)
        if not args.no_batched:
            progress("batched 64 boxes vs sequential")
            v["batched"] = batched(args)
        out["variants"] = v
    if args.paper_spreading:
        out["paper_spreading"] = paper_spreading(
            [float(t) for t in args.paper_spreading.split(",")], args.paper_tmu)
    if args.paper_sec4:
        out["paper_sec4"] = paper_sec4(*args.paper_sec4_tmu)
    if args.paper_shear > 0:
        out["paper_shear"] = paper_shear(args.paper_shear)
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
