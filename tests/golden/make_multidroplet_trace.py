"""Write the FP64 oracle's observable trace of the 512x512x256 box with 16
droplets (the largest single-GPU workload: 67,108,864 cells, 163,872 nodes)
every `every` steps up to `steps`, per droplet and for the box.  The file is
rewritten after each row, so a run cut short leaves the rows it reached.
Calls only the oracle and the input generators.

    python tests/golden/make_multidroplet_trace.py [steps] [every]
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

KEYS = ("height", "contact_radius", "volume", "area", "z_min", "z_max", "cx", "cy", "cz")


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 525
    every = int(sys.argv[2]) if len(sys.argv) > 2 else 25
    wl = configs.multidroplet_c5()
    sim = oracle.OracleSim(wl)
    rows = []
    t0 = time.time()
    path = os.path.join(HERE, "multidroplet_trace_oracle.json")
    while sim.step_count < steps:
        sim.step(every)
        drops, boxes = sim.observables()
        rows.append({"step": sim.step_count, "mass": boxes[0]["mass"], "max_u": boxes[0]["max_u"],
                     "droplets": [{k: d[k] for k in KEYS} for d in drops]})
        out = {"workload": wl.name, "workload_sha256": workload_hash(wl), "every": every,
               "steps": sim.step_count, "oracle_threads": oracle.num_threads(), "rows": rows}
        with open(path + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1)
        os.replace(path + ".tmp", path)
        print(f"step {sim.step_count} h0={drops[0]['height']:.6f} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
