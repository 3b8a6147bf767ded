"""The paper's own spreading runs at their scale on the GPU.

Sec. 3, Fig. 2: 250 x 250 x 150 lattice, a 118,580-triangle mesh, R0 = 60,
90 -> 60 deg.  The boundary element data of the paper are not available,
so this is the self-consistency check the paper allows: the Stokes-limit
height h / R0 of about 0.96 (tests/golden/paper_spreading_sec3.txt) and, at
the highest Reynolds number of the paper (tau = 0.56, Re = 150), the drop
below the final height followed by a recovery that the paper describes.

Sec. 4, inertial case (tests/golden/paper_spreading_sec4.txt): a sphere
released next to the wall first touches it through a neck that widens while
the droplet keeps its full height."""
import math
import os

import pytest

from iblb_inputs import configs

from _helpers import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_spreading_sec3.txt")
GOLDEN4 = os.path.join(os.path.dirname(__file__), "golden", "paper_spreading_sec4.txt")


def _golden(path=GOLDEN):
    out = {}
    for line in open(path):
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


def test_paper_scale_sphere_touches_the_wall_through_a_neck():
    # measured over the first 6 t_mu: r_c / R0 0.381 -> 0.750 while h / R0
    # stays at 2.000 -> 1.994; at 3 t_mu the cross-section 1/24 of the
    # height above the lowest node has 0.58 of the widest radius.  (The
    # whole run, bench.py --paper-sec4: the droplet flattens quickly after
    # about 20 t_mu, falls to h / R0 = 0.684 at 35 t_mu and recovers to 0.716
    # with an apparent angle of 44.7 deg at 50 t_mu.)
    from bench import half_profile
    g = _golden(GOLDEN4)
    import paper_2604_17463_amd as P
    say("paper-scale sphere at the wall, tau 0.56")
    wl = configs.paper_neck()
    b, d0 = wl.boxes[0], wl.droplets[0]
    assert (b.nx, b.ny, b.nz) == tuple(int(v) for v in g["NECK_LATTICE"])
    assert abs(b.tau - g["NECK_TAU"][0]) < 1e-12
    assert abs(math.degrees(d0.theta_eq) - g["THETA_EQ_DEG"][0]) < 1e-9
    assert abs(d0.xi / wl.extra["r0"] - g["XI_OVER_R0"][0]) < 1e-12
    assert abs(d0.nodes[:, 2].min() - d0.xi) < 1e-9
    s = P.Simulation(wl, storage=1, flags=1 | 2)
    tmu, r0 = wl.extra["t_mu"], wl.extra["r0"]
    v0 = s.observables()[0][0]["volume"]
    rc, h = [], []
    for k in range(6):
        s.step(int(round(tmu)))
        d = s.observables()[0][0]
        rc.append(d["contact_radius"] / r0)
        h.append(d["height"] / r0)
        if k == 2:
            prof = half_profile(s.read_nodes(0), d0.tris, d["cx"], d["cy"], levels=12)
    assert all(r1 > r0_ for r0_, r1 in zip(rc, rc[1:]))      # the neck widens
    assert 0.3 < rc[0] < 0.5 and rc[-1] > 0.65
    assert min(h) > 1.98                                     # still at full height
    radii = [r for _, r in prof]
    assert radii[0] < 0.7 * max(radii)                       # a neck at the wall
    assert abs(d["volume"] / v0 - 1.0) < 2e-3
    s.close()


def test_paper_scale_forces_spread_and_step_match_oracle():
    # oracle parity at the scale of the paper's runs: after 300 GPU steps of
    # the 250 x 250 x 150 / 118,580-triangle run (tau = 0.732), on the GPU's
    # own node positions, the nodal forces (2e-5 of the largest), the spread
    # force field over all 9.4 M cells (relative L2 1e-6) and the stamped
    # tiles (bit-exact); then the GPU's next step against the oracle's step
    # from the GPU's state (deviations 1e-5, nodes 1e-6 lu, mass 1e-9)
    import numpy as np

    import oracle
    import paper_2604_17463_amd as P
    from _helpers import deviation, lib_to_oracle_perm, rel_l2, to_oracle
    say("paper-scale forces, spread and one step against the oracle")
    wl = configs.paper_spreading(0.732)
    box, dr = wl.boxes[0], wl.droplets[0]
    shape = (box.nz, box.ny, box.nx)
    s = P.Simulation(wl, storage=1, flags=1)
    s.step(300)
    q = s.read_nodes(0)
    A = oracle.wetting_A(dr.sigma, dr.theta_eq, dr.xi, dr.n_exp, dr.m_exp)
    want = oracle.node_forces(dr.tris, q, dr.sigma, A, dr.xi, dr.n_exp, dr.m_exp, dr.k_vol,
                              oracle.volume(dr.tris, dr.nodes))["phi"]
    got = s.compute_forces(0)
    assert np.abs(got - want).max() < 2e-5 * np.abs(want).max()
    F, flags = s.compute_spread(0)
    Fo, _ = oracle.spread(shape, box.zbc, q, got)
    assert rel_l2(F, Fo) < 1e-6
    assert np.array_equal(flags, oracle.touched_tiles(q, shape, box.zbc, tile=P.band_tile()))
    del F, Fo
    perm = lib_to_oracle_perm()
    f0 = to_oracle(s.read_state(0), perm)
    ref = oracle.OracleSim(wl, f0=[f0])
    ref.q[0] = q.copy()
    ref.step(1)
    s.step(1)
    f1 = to_oracle(s.read_state(0), perm)
    assert rel_l2(deviation(f1), deviation(ref.f[0])) < 1e-5
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-6
    _, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    assert abs(boxes[0]["mass"] - oracle.mass(ref.f[0])) < 1e-9 * oracle.mass(ref.f[0])


def test_paper_neck_step_matches_oracle_from_gpu_state():
    # the Sec. 4 sphere released at the wall at its scale (300 x 300 x 250,
    # R0 = 60, tau = 0.56, the lowest nodes at xi above the wall where the
    # neck forms): after 300 GPU steps, the oracle's step from the GPU's
    # populations and nodes against the GPU's next step (deviations 1e-5
    # relative L2, nodes 1e-6 lu, mass 1e-9)
    import numpy as np

    import oracle
    import paper_2604_17463_amd as P
    from _helpers import deviation, lib_to_oracle_perm, rel_l2, to_oracle
    say("paper-scale neck run: one step against the oracle")
    wl = configs.paper_neck()
    s = P.Simulation(wl, storage=1, flags=1)
    s.step(300)
    perm = lib_to_oracle_perm()
    f0 = to_oracle(s.read_state(0), perm)
    q0 = s.read_nodes(0)
    s.step(1)
    _, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    f1 = to_oracle(s.read_state(0), perm)
    q1 = s.read_nodes(0)
    s.close()
    ref = oracle.OracleSim(wl, f0=[f0])
    del f0
    ref.q[0] = q0.copy()
    ref.step(1)
    assert ref.below_wall == 0
    err_f = rel_l2(deviation(f1), deviation(ref.f[0]))
    err_q = np.abs(q1 - ref.q[0]).max()
    say(f"populations {err_f:.3e}, nodes {err_q:.3e} lu")
    assert err_f < 1e-5, err_f
    assert err_q < 1e-6, err_q
    assert abs(boxes[0]["mass"] - oracle.mass(ref.f[0])) < 1e-9 * oracle.mass(ref.f[0])
