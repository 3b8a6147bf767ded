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
