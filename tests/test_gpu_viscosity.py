"""GPU parity of the viscosity contrast (paper Sec. 2, below Eq. 13: cells
inside the droplets relax with tau_in, found by ray tracing) against the
FP64 oracle, through the C ABI.

The inside bits are integer work: bit-exact against the oracle's inside test
on the positions the GPU holds.  Whole steps with tau_in: the same
tolerances as the single-viscosity steps (FP64 1e-10 relative L2, FP32
1e-5 on velocities); graph replay bitwise equal to eager launches."""
import numpy as np
import pytest

import oracle
from iblb_inputs import configs, mesh
from iblb_inputs.configs import Box, Droplet, Workload

from _helpers import deviation, lib_to_oracle_perm, rel_l2, say, to_oracle

pytestmark = pytest.mark.gpu

F64, F32, F16 = 0, 1, 2
FULL_U, GRAPH = 4, 1


def sim(wl, storage, flags=0):
    import paper_2604_17463_amd as P
    return P.Simulation(wl, storage=storage, flags=flags,
                        dev_scale=4096.0 if storage == F16 else 1.0)


@pytest.fixture(scope="module")
def perm():
    return lib_to_oracle_perm()


def _box_mesh(lo, hi):
    v = np.array([[(lo[0], hi[0])[x], (lo[1], hi[1])[y], (lo[2], hi[2])[z]]
                  for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=float)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return v, np.array(t, dtype=np.int32)


def _drop(box, v, t):
    return Droplet(box, v, t, sigma=0.01, theta_eq=np.pi / 2, xi=0.4, k_vol=0.0)


def _oracle_inside(s, wl, b):
    """The oracle's inside test of box b on the node positions the GPU holds."""
    bx = wl.boxes[b]
    tris, qs, off = [], [], 0
    for d, dr in enumerate(wl.droplets):
        if dr.box != b:
            continue
        tris.append(np.asarray(dr.tris, np.int32) + off)
        q = s.read_nodes(d)
        qs.append(q)
        off += len(q)
    return oracle.inside((bx.nz, bx.ny, bx.nx), np.concatenate(tris), np.concatenate(qs))


def _c1_contrast(tau_in=1.6, jitter=None):
    wl = configs.plain_c1()
    wl.boxes[0].tau_in = tau_in
    if jitter is not None:
        d = wl.droplets[0]
        d.nodes = configs.jitter_nodes(d.nodes, jitter, 0.2)
    return wl


def _cases():
    # jittered sphere above the wall
    yield "c1-jittered", _c1_contrast(jitter=3)
    # faces on cell-centre planes and triangle edges through cell centres:
    # every cell of the box's columns meets the tie rule
    v, t = _box_mesh((2.5, 2.5, 2.5), (6.5, 6.5, 6.5))
    yield "box-ties", Workload("ties", [Box(10, 10, 10, tau=0.8, tau_in=1.2)],
                               [_drop(0, v, t)], storage=F64)
    # two droplets, one across the periodic x side (nodes unwrapped past nx),
    # with a mask column height nz = 70 that spans two 64-bit words
    v1, t1 = mesh.sphere(3, 5.0, (31.0, 12.0, 40.0))
    v2, t2 = mesh.sphere(3, 4.0, (14.0, 11.5, 62.5))
    v3, t3 = mesh.sphere(3, 6.0, (12.0, 14.0, 8.0))
    v3 = configs.jitter_nodes(v3, 5, 0.3)
    yield "multi-periodic", Workload(
        "multi", [Box(32, 24, 70, tau=0.7, zbc=1, tau_in=1.1)],
        [_drop(0, v1, t1), _drop(0, v2, t2), _drop(0, v3, t3)], storage=F64)


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("case", ["c1-jittered", "box-ties", "multi-periodic"])
def test_inside_bits_match_oracle(case, storage):
    say("inside bits", case, storage)
    wl = dict(_cases())[case]
    s = sim(wl, storage)
    got = s.read_inside(0)
    want = _oracle_inside(s, wl, 0)
    assert want.sum() > 0
    assert np.array_equal(got, want)
    if case == "box-ties":
        assert got.sum() == 64
    # and again after the nodes moved
    s.step(5)
    assert np.array_equal(s.read_inside(0), _oracle_inside(s, wl, 0))


def test_inside_bits_follow_written_nodes():
    say("inside bits after write_nodes")
    wl = _c1_contrast()
    s = sim(wl, F64)
    q = s.read_nodes(0) + np.array([3.25, -2.5, 1.0])
    s.write_nodes(q)
    got = s.read_inside(0)
    assert np.array_equal(got, _oracle_inside(s, wl, 0))


def test_read_inside_rejects_a_box_without_tau_in():
    say("read_inside without tau_in")
    s = sim(configs.plain_c1(), F64)
    with pytest.raises(RuntimeError):
        s.read_inside(0)


def test_contrast_c1_fp64_full_parity(perm):
    say("contrast c1 fp64 200 steps")
    wl = _c1_contrast()
    s = sim(wl, F64, flags=FULL_U)
    ref = oracle.OracleSim(wl)
    ref.step(200)
    s.step(200)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    assert rel_l2(u, ref.last_u[0]) < 1e-10
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-10
    # every cell whose inside bit changed lay in the band
    _, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    # the contrast changes the run: a single-viscosity run differs
    plain = oracle.OracleSim(configs.plain_c1())
    plain.step(200)
    assert rel_l2(u, plain.last_u[0]) > 1e-3


def test_contrast_fp32_and_mixed_boxes_parity(perm):
    # box 0 has a contrast, box 1 (same droplet shifted) has none: the
    # library's per-box selection against the oracle's
    say("contrast fp32 two boxes 120 steps")
    a = _c1_contrast(tau_in=0.7)
    b = configs.plain_c1()
    d1 = b.droplets[0]
    d1.nodes = d1.nodes + np.array([1.3, -0.6, 0.0])
    d1.box = 1
    wl = Workload("mixed", [a.boxes[0], b.boxes[0]], [a.droplets[0], d1], storage=F32)
    s = sim(wl, F32, flags=FULL_U)
    ref = oracle.OracleSim(wl)
    ref.step(120)
    s.step(120)
    for bi in range(2):
        f, u = s.read_state(bi, want_u=True)
        f = to_oracle(f, perm)
        assert rel_l2(f, ref.f[bi]) < 1e-6, bi
        assert rel_l2(u, ref.last_u[bi]) < 1e-5, bi
        assert np.abs(s.read_nodes(bi) - ref.q[bi]).max() < 1e-5, bi


def test_band_after_bulk_schedule_is_refused_with_a_viscosity_contrast():
    # that schedule relaxes the cells outside the band with the previous
    # step's inside bits; with tau_in only the exact schedule is allowed
    import paper_2604_17463_amd as P
    say("schedule refused with tau_in")
    s = sim(_c1_contrast(), F32)
    with pytest.raises(P.IblbError) as e:
        s.set_launch(64, 4, 1, 0, 0, 1)
    assert e.value.code == -1
    s.set_launch(64, 4, 1, 0, 0, 0)
    s.step(2)


@pytest.mark.parametrize("storage", [F32, F16])
def test_contrast_graph_replay_is_bitwise_equal_to_eager(storage):
    say("contrast graph vs eager", storage)
    wl = _c1_contrast()
    a = sim(wl, storage, flags=0)
    b = sim(wl, storage, flags=GRAPH)
    a.step(37)
    b.step(37)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))
    assert np.array_equal(a.read_inside(0), b.read_inside(0))


def test_inside_change_away_from_the_stencils_follows_the_oracle():
    # An 8-node cube of side 16 carried by a body-force driven flow: its
    # x = lo face crosses the cell centres x = 8.5 mid-face, 8 lu from every
    # node, so those cells change status outside every stamped tile.  Every
    # cell relaxes with the inside bits of its own step (the stream-collide
    # of the cells outside the band runs after the step's inside test), so
    # the run matches the oracle to the FP64 tolerance and raises no status
    # bit.
    say("inside change outside the band, FP64 against the oracle")
    v, t = _box_mesh((8.45, 8.0, 8.0), (24.45, 24.0, 24.0))
    d = Droplet(0, v, t, sigma=1e-5, theta_eq=np.pi, xi=0.4, k_vol=0.0)
    wl = Workload("cube", [Box(40, 32, 32, tau=0.8, zbc=1, body_force=(2e-4, 0.0, 0.0),
                               tau_in=1.2)], [d], storage=F64)
    s = sim(wl, F64)
    before = s.read_inside(0)
    assert before[16, 16, 8] == 1
    ref = oracle.OracleSim(wl)
    ref.step(60)
    s.step(60)
    after = s.read_inside(0)
    assert after[16, 16, 8] == 0
    assert np.array_equal(after, ref.inside_mask(0).astype(after.dtype))
    perm = lib_to_oracle_perm()
    f = to_oracle(s.read_state(0), perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-10
    _, boxes = s.observables(raise_unstable=False)
    assert boxes[0]["status_bits"] == 0
