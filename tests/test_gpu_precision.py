"""Precision workload (256x256x128 box, one 40,962-node sphere of radius 48
relaxing toward 45 degrees, tau = 0.6 and 1.0) against the FP64 oracle's
stored trace at 2,000 steps, for each population storage.

FP64 and FP32 storage are held to the trace-parity bounds of the spreading
run (height 1e-4, contact radius 1e-3, volume 1e-6, mass 1e-8 relative).
FP16 and BF16 deviation storage carry their own rounding (11 and 8
significant bits of each stored deviation, FP32 arithmetic); their errors
are reported, and bounded only loosely (height 1e-3, contact radius 2e-2,
volume 1e-4, mass 1e-5), so that a broken conversion still fails.
"""
import json
import os
import sys

import pytest

from _helpers import say

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

KEYS = ("height", "contact_radius", "volume", "mass")
TIGHT = {"height": 1e-4, "contact_radius": 1e-3, "volume": 1e-6, "mass": 1e-8}
LOOSE = {"height": 1e-3, "contact_radius": 2e-2, "volume": 1e-4, "mass": 1e-5}


@pytest.mark.gpu
@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_precision_workload_against_oracle_trace(tau):
    import paper_2604_17463_amd as P
    from iblb_inputs import configs
    from make_spreading_trace import workload_hash

    with open(os.path.join(HERE, "golden", f"precision_trace_oracle_tau{tau:g}.json")) as fh:
        tr = json.load(fh)
    steps = tr["steps"]
    wl = configs.precision_c3(tau=tau, steps=steps)
    assert tr["workload_sha256"] == workload_hash(wl), "stored trace is of another workload"
    ref = {r["step"]: r for r in tr["rows"]}[steps]
    report = {}
    for storage, name, bound in ((P.IBLB_F64, "f64", TIGHT), (P.IBLB_F32, "f32", TIGHT),
                                 (P.IBLB_F16DEV, "f16dev", LOOSE), (P.IBLB_BF16DEV, "bf16dev", LOOSE)):
        say(f"precision workload tau {tau}: {name}, {steps} steps")
        sim = P.Simulation(wl, storage=storage, flags=P.IBLB_FLAG_GRAPH,
                           dev_scale=4096.0 if storage == P.IBLB_F16DEV else 1.0)
        sim.step(steps)
        d, b = sim.observables()
        sim.close()
        got = {"height": d[0]["height"], "contact_radius": d[0]["contact_radius"],
               "volume": d[0]["volume"], "mass": b[0]["mass"]}
        err = {k: abs(got[k] - ref[k]) / abs(ref[k]) for k in KEYS}
        report[name] = err
        for k in KEYS:
            assert err[k] <= bound[k], f"{name} {k}: {err[k]:.3e} > {bound[k]:.0e}"
    say("relative errors vs oracle: " + json.dumps(report))
