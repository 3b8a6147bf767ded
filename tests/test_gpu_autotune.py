"""The autotuner's results are kept: a second init of the same configuration
in the process takes the first one's launch without timing again, and a
launch stored in the file named by IBLB_TUNE_CACHE is taken by a fresh
process.  Whatever launch a context runs with, the results are those of the
default launch bit for bit."""
import json
import os
import subprocess
import sys
import time

import numpy as np
import pytest

from iblb_inputs import configs

from _helpers import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GRAPH, AUTOTUNE = 1, 2


def test_second_init_reuses_the_tuned_launch():
    import paper_2604_17463_amd as P
    from iblb_inputs.configs import Box, Workload
    say("autotune kept in the process")
    # a box size no other test tunes, so that the first init here times the
    # candidates whatever ran before in the process
    c1 = configs.plain_c1()
    b0 = c1.boxes[0]
    wl = Workload("autotune-keep", [Box(b0.nx + 8, b0.ny, b0.nz, tau=b0.tau)], c1.droplets, storage=c1.storage)
    t0 = time.perf_counter()
    a = P.Simulation(wl, storage=1, flags=GRAPH | AUTOTUNE)
    t1 = time.perf_counter()
    b = P.Simulation(wl, storage=1, flags=GRAPH | AUTOTUNE)
    t2 = time.perf_counter()
    assert a.get_launch() == b.get_launch()
    assert t2 - t1 < 0.5 * (t1 - t0), (t1 - t0, t2 - t1)
    ref = P.Simulation(wl, storage=1, flags=GRAPH)
    for s in (a, b, ref):
        s.step(25)
    assert np.array_equal(a.read_state(0), ref.read_state(0))
    assert np.array_equal(b.read_nodes(0), ref.read_nodes(0))


_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import paper_2604_17463_amd as P
from iblb_inputs import configs
wl = configs.spreading_c2()
s = P.Simulation(wl, storage=1, flags=1 | 2)
print(json.dumps(list(s.get_launch())))
"""


def test_tune_cache_file_is_read_by_a_fresh_process(tmp_path):
    say("autotune cache file across processes")
    path = str(tmp_path / "tune.txt")
    env = dict(os.environ, IBLB_TUNE_CACHE=path)
    code = _CHILD.format(root=ROOT)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    tuned = json.loads(r.stdout.strip().splitlines()[-1])
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[1].split() == [str(v) for v in tuned]
    # a different (valid) launch for the same key: a fresh process must take it
    key = lines[0].split("\t")[0]
    forced = [64, 4, 1, 0, 7, 1 - tuned[5]]
    with open(path, "a") as fh:
        fh.write(key + "\t" + " ".join(str(v) for v in forced) + "\n")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert json.loads(r.stdout.strip().splitlines()[-1]) == forced
