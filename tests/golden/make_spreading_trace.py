"""Write the FP64 oracle's observable trace of the 128x128x64 spreading run
(10,242-node cap relaxing from 150 toward 60 degrees, tau = 0.8) every 100
steps up to 20,000 steps.  Calls only the oracle and the input generators.

    python tests/golden/make_spreading_trace.py [steps] [every]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from iblb_inputs import configs  # noqa: E402
from iblb_inputs.configs import workload_hash  # noqa: E402


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 20000
    every = int(sys.argv[2]) if len(sys.argv) > 2 else 100
    wl = configs.spreading_c2(steps=steps)
    sim = oracle.OracleSim(wl)
    rows = []
    t0 = time.time()

    def record():
        drops, boxes = sim.observables()
        d = drops[0]
        rows.append({"step": sim.step_count, "height": d["height"],
                     "contact_radius": d["contact_radius"], "volume": d["volume"],
                     "area": d["area"], "z_min": d["z_min"], "z_max": d["z_max"],
                     "cx": d["cx"], "cy": d["cy"], "cz": d["cz"],
                     "n_crossings": d["n_crossings"], "mass": boxes[0]["mass"],
                     "max_u": boxes[0]["max_u"]})

    record()
    while sim.step_count < steps:
        sim.step(every)
        record()
        print(f"step {sim.step_count} h={rows[-1]['height']:.6f} "
              f"rc={rows[-1]['contact_radius']:.6f} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": wl.name, "workload_sha256": workload_hash(wl), "every": every,
           "steps": steps, "oracle_threads": oracle.num_threads(), "rows": rows}
    with open(os.path.join(HERE, "spreading_trace_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
