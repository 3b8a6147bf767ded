"""The paper's own spreading run at its scale (Sec. 3, Fig. 2) on the GPU:
250 x 250 x 150 lattice, a 118,580-triangle mesh, R0 = 60, 90 -> 60 deg.
The boundary element data of the paper are not available, so this is the
self-consistency check the paper allows: the Stokes-limit height h / R0
of about 0.96 (tests/golden/paper_spreading_sec3.txt) and, at the highest
Reynolds number of the paper (tau = 0.56, Re = 150), the drop below the
final height followed by a recovery that the paper describes."""
import math
import os

import pytest

from iblb_inputs import configs

from _helpers import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_spreading_sec3.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *v = line.split()
            out[k] = [float(x) for x in v]
    return out


def test_paper_scale_spreading_at_re_150():
    # measured: h / R0 falls to 0.910 near 30 t_mu and recovers to 0.929 at
    # 50 t_mu; apparent angle 62.2 deg; volume kept to 5e-4.  (The Stokes
    # limit, tau = 1.1 over 600,000 steps, ends at 0.955: bench.py
    # --paper-spreading.)
    g = _golden()
    import paper_2604_17463_amd as P
    say("paper-scale spreading tau 0.56")
    wl = configs.paper_spreading(0.56)
    assert len(wl.droplets[0].tris) == 118580
    assert (wl.boxes[0].nx, wl.boxes[0].ny, wl.boxes[0].nz) == tuple(int(v) for v in g["LATTICE"])
    s = P.Simulation(wl, storage=1, flags=1 | 2)
    tmu, r0 = wl.extra["t_mu"], wl.extra["r0"]
    d0 = s.observables()[0][0]
    assert abs(math.degrees(d0["theta_app"]) - g["THETA_START_DEG"][0]) < 1.0
    h = []
    for _ in range(int(g["T_END_OVER_TMU"][0])):
        s.step(int(round(tmu)))
        d = s.observables()[0][0]
        h.append(d["height"] / r0)
    assert abs(h[-1] / g["H_INF_OVER_R0"][0] - 1.0) < 0.04
    assert min(h) < h[-1] - 0.01                       # undershoot, then recovery
    assert abs(math.degrees(d["theta_app"]) - g["THETA_EQ_DEG"][0]) < 3.0
    assert abs(d["volume"] / d0["volume"] - 1.0) < 1e-3
