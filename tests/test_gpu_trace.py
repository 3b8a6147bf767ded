"""Trace parity of the 128x128x64 spreading run (10,242-node ico5 cap
relaxing from 150 toward 60 degrees, tau = 0.8, FP32 storage, graph replay
with the autotuned bulk launch) against the FP64 oracle's stored trace,
every 100 steps up to 20,000 steps.

Bounds (relative, at every logged step):
  height          1e-4
  contact radius  1e-3
  volume          1e-6
  mass            1e-8
The FP32 path rounds every stored population deviation once per step; the
rounding errors of ~1e6 cells x 19 populations do not cancel exactly, so
the total mass walks away from the exactly conserved FP64 value by about
2e-9 per 5,000 steps (measured); 1e-8 bounds that drift over 20,000 steps
while still catching any non-conserving update (a single unbalanced
population per cell and step would move it by >1e-4).
"""
import json
import os
import sys

import pytest

from _helpers import say

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

TOL = {"height": 1e-4, "contact_radius": 1e-3, "volume": 1e-6, "mass": 1e-8}


@pytest.mark.gpu
def test_spreading_trace_fp32_matches_the_oracle_every_100_steps():
    import paper_2604_17463_amd as P
    from iblb_inputs import configs
    from iblb_inputs.configs import workload_hash

    with open(os.path.join(HERE, "golden", "spreading_trace_oracle.json")) as fh:
        tr = json.load(fh)
    wl = configs.spreading_c2(steps=tr["steps"])
    assert tr["workload_sha256"] == workload_hash(wl), "stored trace is of another workload"
    say("spreading trace: FP32, graph + autotune, 20k steps")
    sim = P.Simulation(wl, storage=P.IBLB_F32, flags=P.IBLB_FLAG_GRAPH | P.IBLB_FLAG_AUTOTUNE)
    worst = {k: (0.0, 0) for k in TOL}
    done = 0
    for row in tr["rows"]:
        if row["step"] > done:
            sim.step(row["step"] - done)
            done = row["step"]
        drops, boxes = sim.observables()
        d, b = drops[0], boxes[0]
        assert d["step"] == row["step"]
        got = {"height": d["height"], "contact_radius": d["contact_radius"],
               "volume": d["volume"], "mass": b["mass"]}
        for k in TOL:
            e = abs(got[k] - row[k]) / abs(row[k])
            if e > worst[k][0]:
                worst[k] = (e, row["step"])
    say("worst relative errors (error, step): " + json.dumps(worst))
    sim.close()
    for k, (e, st) in worst.items():
        assert e <= TOL[k], f"{k}: {e:.3e} at step {st} > {TOL[k]:.0e}"


# Reduced-precision storage of the deviations (FP16 scaled by 4096, BF16) on
# the same trace.  Measured worst relative errors over the 20,000 steps:
#   FP16  height 1.6e-5, contact radius 9.5e-6, volume 1.4e-5, mass 6.4e-7
#   BF16  height 3.2e-3, contact radius 9.0e-4, volume 1.4e-4, mass 2.5e-6
# (BF16 keeps 8 significant bits of each deviation).  The bounds are about
# three times these: regression bounds for the storage formats, reported
# against the FP64 oracle as the method's own error.
TOL_LOWP = {
    "f16dev": {"height": 5e-5, "contact_radius": 3e-5, "volume": 5e-5, "mass": 2e-6},
    "bf16dev": {"height": 1e-2, "contact_radius": 3e-3, "volume": 5e-4, "mass": 1e-5},
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["f16dev", "bf16dev"])
def test_spreading_trace_reduced_precision_matches_the_oracle(name):
    import paper_2604_17463_amd as P
    from iblb_inputs import configs
    from iblb_inputs.configs import workload_hash

    with open(os.path.join(HERE, "golden", "spreading_trace_oracle.json")) as fh:
        tr = json.load(fh)
    wl = configs.spreading_c2(steps=tr["steps"])
    assert tr["workload_sha256"] == workload_hash(wl), "stored trace is of another workload"
    storage, scale = (P.IBLB_F16DEV, 4096.0) if name == "f16dev" else (P.IBLB_BF16DEV, 1.0)
    say(f"spreading trace: {name}, graph + autotune, 20k steps")
    sim = P.Simulation(wl, storage=storage, flags=P.IBLB_FLAG_GRAPH | P.IBLB_FLAG_AUTOTUNE,
                       dev_scale=scale)
    tol = TOL_LOWP[name]
    worst = {k: (0.0, 0) for k in tol}
    done = 0
    for row in tr["rows"]:
        if row["step"] > done:
            sim.step(row["step"] - done)
            done = row["step"]
        drops, boxes = sim.observables()
        d, b = drops[0], boxes[0]
        got = {"height": d["height"], "contact_radius": d["contact_radius"],
               "volume": d["volume"], "mass": b["mass"]}
        for k in tol:
            e = abs(got[k] - row[k]) / abs(row[k])
            if e > worst[k][0]:
                worst[k] = (e, row["step"])
    say("worst relative errors (error, step): " + json.dumps(worst))
    sim.close()
    for k, (e, st) in worst.items():
        assert e <= tol[k], f"{name} {k}: {e:.3e} at step {st} > {tol[k]:.0e}"
