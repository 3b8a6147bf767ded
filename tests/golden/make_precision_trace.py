"""Write the FP64 oracle's observable trace of the 256x256x128 precision
workload (one 40,962-node sphere of radius 48 relaxing toward 45 degrees)
for tau = 0.6 and tau = 1.0, every 500 steps up to the workload's configured
10,000 steps.  Calls only the oracle and the input generators.

    python tests/golden/make_precision_trace.py [steps] [every]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from iblb_inputs import configs  # noqa: E402
from iblb_inputs.configs import workload_hash  # noqa: E402


def trace(tau, steps, every):
    wl = configs.precision_c3(tau=tau, steps=steps)
    sim = oracle.OracleSim(wl)
    rows = []
    t0 = time.time()

    def record():
        drops, boxes = sim.observables()
        d = drops[0]
        rows.append({"step": sim.step_count, "height": d["height"],
                     "contact_radius": d["contact_radius"], "volume": d["volume"],
                     "area": d["area"], "z_min": d["z_min"], "z_max": d["z_max"],
                     "mass": boxes[0]["mass"], "max_u": boxes[0]["max_u"]})

    record()
    while sim.step_count < steps:
        sim.step(every)
        record()
        print(f"tau {tau} step {sim.step_count} h={rows[-1]['height']:.6f} "
              f"rc={rows[-1]['contact_radius']:.6f} ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": wl.name, "workload_sha256": workload_hash(wl), "every": every,
            "steps": steps, "oracle_threads": oracle.num_threads(), "rows": rows}


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 10000
    every = int(sys.argv[2]) if len(sys.argv) > 2 else 500
    for tau in (0.6, 1.0):
        out = trace(tau, steps, every)
        with open(os.path.join(HERE, f"precision_trace_oracle_tau{tau:g}.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
