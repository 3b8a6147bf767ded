"""The bench on the CPU: the HBM bytes it reports as `traffic` come from the
committed counter record's entry for the launch shape the run uses, and from
no other workload, storage or shape; and it refuses any GPU count but one."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

WL = "multidroplet-512x512x256-16xico5"


def _record():
    with open(bench.TRAFFIC) as fh:
        return json.load(fh)


def test_traffic_follows_the_launch_shape_of_the_run():
    rec = _record()
    entries = [rec] + rec["launches"]
    shapes = [tuple(e["launch"][:5]) for e in entries]
    assert len(set(shapes)) == len(shapes)
    for e in entries:
        # the step schedule (sixth field) does not change the bulk kernel
        for after in (0, 1):
            got = bench.counted_traffic(rec, WL, "f32", list(e["launch"][:5]) + [after])
            assert got == e["hbm_bytes_per_launch"]
    assert bench.counted_traffic(rec, WL, "f32", [64, 4, 1, 1, 0, 0]) is None
    assert bench.counted_traffic(rec, WL, "f16dev", list(rec["launch"])) is None
    assert bench.counted_traffic(rec, "box-256x256x128", "f32", list(rec["launch"])) is None
    assert bench.counted_traffic(None, WL, "f32", list(rec["launch"])) is None


def test_record_entries_are_consistent():
    rec = _record()
    f, w = rec["calibration"]["fetch_factor"], rec["calibration"]["write_factor"]
    alg = 67108864 * bench.cell_bytes("f32")
    for e in [rec] + rec["launches"]:
        hbm = 1024 * (e["fetch_KiB_per_launch_raw"] * f + e["write_KiB_per_launch_raw"] * w)
        assert abs(hbm - e["hbm_bytes_per_launch"]) < 1e-4 * hbm
        assert e["algorithmic_bytes_per_launch"] == alg
        # every population is read and written at least once per launch
        assert 1.0 <= e["hbm_bytes_per_launch"] / alg < 1.05


def test_bench_refuses_several_gpus():
    # one GPU only: any other count exits before touching a device
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _headline_trace():
    with open(bench.MTRACE) as fh:
        return json.load(fh)


def test_headline_oracle_trace_is_of_the_headline_workload():
    # written by tests/golden/make_multidroplet_trace.py (oracle only): the
    # inputs it was made from are those the bench runs, its rows lie every
    # 25 steps from step 25 (where the driver's 5 + 20 steps end), and the
    # closed box keeps its mass to rounding
    from iblb_inputs import configs
    tr = _headline_trace()
    wl = configs.multidroplet_c5()
    assert tr["workload_sha256"] == configs.workload_hash(wl)
    steps = [r["step"] for r in tr["rows"]]
    assert steps == list(range(25, 25 * len(steps) + 1, 25))
    for r in tr["rows"]:
        assert abs(r["mass"] - wl.cells) < 1e-9 * wl.cells
        assert len(r["droplets"]) == len(wl.droplets)


class _StandIn:
    """Reports the stored trace's values at whatever step it has reached."""

    def __init__(self, tr, step):
        self.rows = {r["step"]: r for r in tr["rows"]}
        self.now = step

    def step(self, n):
        self.now += n

    def observables(self):
        r = self.rows.get(self.now)
        drops = [dict(d, step=self.now) for d in (r["droplets"] if r else [{}])]
        return drops, [{"step": self.now, "mass": r["mass"] if r else 0.0}]


def test_headline_error_is_taken_at_the_next_trace_row():
    from iblb_inputs import configs
    tr = _headline_trace()
    wl = configs.multidroplet_c5()
    sim = _StandIn(tr, 20)
    out = bench.headline_oracle_errors(sim, wl)
    assert out["step"] == 25 and sim.now == 25
    assert all(out[k] == 0.0 for k in ("height", "contact_radius", "volume", "area", "mass"))
    last = tr["rows"][-1]["step"]
    assert bench.headline_oracle_errors(_StandIn(tr, last + 1), wl) is None
    other = configs.multidroplet_c5(seed=1)
    assert bench.headline_oracle_errors(_StandIn(tr, 20), other) is None
