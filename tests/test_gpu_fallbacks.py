"""GPU parity of the kernels' fallback paths, through the C ABI, each on a
workload built so that the path is certainly taken (the condition is checked
on the node positions in the test):

  - a node block whose stencil box exceeds the 2,048-cell partial-spread
    region: its force is summed node by node in the band gather, and the
    interpolation reads the band velocities from memory instead of an LDS
    stage (the region exceeds the stage);
  - a band tile covered by more than the 16 node blocks a tile records:
    the gather tests every block's bounding box instead;
  - a box whose node block covers more than 64 band tiles along an axis:
    the tile records of the whole box are abandoned for the scan.

Each is checked against the FP64 oracle element by element: the spread force
(relative L2 1e-13 in FP64, 1e-6 in FP32) and the stamped tiles (bit-exact),
the interpolation of a seeded velocity field (1e-13 / 1e-6), and in FP64 ten
whole steps (populations and nodes within 1e-10).

Also the status word: a node driven below the wetting wall sets the WALL bit,
and a node put beyond |q| = 1e7 sets the JUMP bit; both turn
iblb_observables into IBLB_E_UNSTABLE and refuse further steps.  Reading the
node pass and the interpolation for d <= 0: the base cell floor(q - 1/2) is
then -1 or below, stencil cells in the wall are not stamped and their spread
weight is dropped (the region's z range is clipped to [0, nz)), and the
interpolation reads only cells with 0 <= z < nz, so every access stays in
the box.
"""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import configs, mesh
from iblb_inputs.configs import Box, Droplet, Workload

from _helpers import deviation, lib_to_oracle_perm, rel_l2, say, to_oracle

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1
GRAPH = 1
NB = 64
MAXP, MAXC, SCAN_GROUP = 2048, 16, 256


def sim(wl, storage, flags=GRAPH):
    import paper_2604_17463_amd as P
    return P.Simulation(wl, storage=storage, flags=flags)


def _stencil_extent(q):
    """Cells of the stencil bounding box of the nodes q (x, y unwrapped, z
    clipped to the fluid is not needed for these lower bounds)."""
    b = np.floor(q - 0.5).astype(int)
    return (b.max(0) + 2) - (b.min(0) - 1) + 1


def _coarse(nz=40):
    # ico1: 42 nodes, one node block, stencil box about 28^3 cells
    r = 12.0
    v, t = mesh.sphere_above_wall(1, r, 24.3, 23.8, 0.05 * r)
    return Workload("coarse", [Box(48, 48, nz, tau=0.9)],
                    [Droplet(0, v, t, sigma=0.01, theta_eq=math.radians(70), xi=0.05 * r,
                             k_vol=2 * 0.01 / r)], storage=F64)


def _dense():
    # ico6 of radius 8: 40,962 nodes (641 blocks) on a surface of ~800 lu^2
    r = 8.0
    v, t = mesh.sphere_above_wall(6, r, 16.4, 18.1, 0.05 * r)
    return Workload("dense", [Box(32, 36, 24, tau=0.8)],
                    [Droplet(0, v, t, sigma=0.01, theta_eq=math.radians(60), xi=0.05 * r)],
                    storage=F64)


def _tall_and_dense():
    # a coarse ico1 of radius 34 (one block spanning about 72 cells in z) and
    # an ico6 of radius 8 in one box: more than 256 blocks, so the box keeps
    # tile records, which the tall block then abandons
    v1, t1 = mesh.sphere_above_wall(1, 34.0, 40.0, 48.0, 1.7)
    v2, t2 = mesh.sphere_above_wall(6, 8.0, 100.2, 47.6, 0.4)
    return Workload("tall", [Box(128, 96, 80, tau=0.9)],
                    [Droplet(0, v1, t1, sigma=0.005, theta_eq=math.radians(80), xi=1.7),
                     Droplet(0, v2, t2, sigma=0.01, theta_eq=math.radians(60), xi=0.4)],
                    storage=F64)


def _check_conditions(name, wl):
    if name == "coarse":
        q = wl.droplets[0].nodes
        assert len(q) <= NB  # one block
        assert np.prod(_stencil_extent(q)) > 3 * MAXP  # beyond the region and the FP32 stage
    elif name == "dense":
        import paper_2604_17463_amd as P
        q = wl.droplets[0].nodes
        box = wl.boxes[0]
        assert len(q) > SCAN_GROUP * NB
        # nodes whose stencil touches each band tile; more than 16 * 64 of
        # them means more than 16 distinct blocks cover the tile
        sx, sy, sz = P.band_tile()
        b = np.floor(q - 0.5).astype(np.int64)
        o = np.arange(-1, 3)
        tx = (b[:, 0, None] + o) % box.nx // sx
        ty = (b[:, 1, None] + o) % box.ny // sy
        tz = (b[:, 2, None] + o + 2) // sz
        ids = (tz[:, :, None, None] * 64 + ty[:, None, :, None]) * 64 + tx[:, None, None, :]
        ids = np.sort(ids.reshape(len(q), -1), axis=1)
        first = np.concatenate([np.ones((len(q), 1), bool), ids[:, 1:] != ids[:, :-1]], axis=1)
        assert np.bincount(ids[first]).max() > MAXC * NB
    else:
        assert sum(len(d.nodes) for d in wl.droplets) > SCAN_GROUP * NB
        assert _stencil_extent(wl.droplets[0].nodes)[2] > 64


CASES = {"coarse": _coarse, "dense": _dense, "tall": _tall_and_dense}


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fallback_spread_and_interpolation_match_oracle(name, storage):
    import paper_2604_17463_amd as P
    say("fallback spread/interp", name, storage)
    wl = CASES[name]()
    _check_conditions(name, wl)
    box = wl.boxes[0]
    s = sim(wl, storage)
    qs = [s.read_nodes(d) for d in range(len(wl.droplets))]
    phis = [s.compute_forces(d) for d in range(len(wl.droplets))]
    F, flags = s.compute_spread(0)
    Fo = np.zeros((3, box.nz, box.ny, box.nx))
    tw = np.zeros(3)
    for q, phi in zip(qs, phis):
        tw += oracle.spread((box.nz, box.ny, box.nx), box.zbc, q, phi, Fo)[1]
    assert rel_l2(F, Fo) < (1e-13 if storage == F64 else 1e-6)
    tile = P.band_tile()
    want = np.zeros_like(flags)
    for q in qs:
        want |= oracle.touched_tiles(q, (box.nz, box.ny, box.nx), box.zbc, tile=tile)
    assert np.array_equal(flags, want)
    total = sum(p.sum(0) for p in phis)
    assert np.allclose(F.sum(axis=(1, 2, 3)) + tw, total, rtol=0,
                       atol=(1e-13 if storage == F64 else 1e-6) * sum(np.abs(p).sum() for p in phis))
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, box.nz, box.ny, box.nx)) * 1e-3
    for d, q in enumerate(qs):
        U = s.interpolate(u, d)
        assert rel_l2(U, oracle.interp(u, box.zbc, q)) < (1e-13 if storage == F64 else 1e-6), d


@pytest.mark.parametrize("name", sorted(CASES))
def test_fallback_steps_match_oracle(name):
    say("fallback whole steps FP64", name)
    wl = CASES[name]()
    perm = lib_to_oracle_perm()
    s = sim(wl, F64)
    ref = oracle.OracleSim(wl)
    s.step(10)
    ref.step(10)
    f = to_oracle(s.read_state(0), perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    for d in range(len(wl.droplets)):
        assert np.abs(s.read_nodes(d) - ref.q[d]).max() < 1e-10, d
    _, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0


def _passive(z_low, g=(0.0, 0.0, 0.0)):
    # a force-free mesh (no surface tension, theta = 180 deg: no wetting
    # amplitude, no volume penalty) carried by the fluid
    v, t = mesh.sphere_above_wall(3, 6.0, 16.2, 15.7, z_low)
    return Workload("passive", [Box(32, 32, 24, tau=0.8, body_force=g)],
                    [Droplet(0, v, t, sigma=0.0, theta_eq=math.pi, xi=0.3)], storage=F32)


def test_node_below_the_wall_sets_the_wall_bit():
    import paper_2604_17463_amd as P
    say("status: node driven through the wetting wall")
    wl = _passive(1e-3, g=(0.0, 0.0, -1e-3))
    s = sim(wl, F32)
    # the host refuses a node placed at or below the wall
    q = s.read_nodes(0)
    bad = q.copy()
    bad[np.argmin(bad[:, 2]), 2] = -1e-3
    with pytest.raises(P.IblbError) as e:
        s.write_nodes(bad)
    assert e.value.code == P.IBLB_E_MESH
    # the downward body force carries the lowest node through z = 0
    bits = 0
    for _ in range(20):
        s.step(2)
        _, boxes = s.observables(raise_unstable=False)
        bits = boxes[0]["status_bits"]
        if bits:
            break
    assert bits & P.IBLB_BIT_WALL, bits
    with pytest.raises(P.IblbError) as e:
        s.observables()
    assert e.value.code == P.IBLB_E_UNSTABLE
    with pytest.raises(P.IblbError) as e:
        s.step(1)
    assert e.value.code == P.IBLB_E_STATE


def test_node_beyond_the_coordinate_range_sets_the_jump_bit():
    import paper_2604_17463_amd as P
    say("status: node beyond |q| = 1e7")
    wl = _passive(3.0)
    s = sim(wl, F32)
    s.step(3)
    _, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    q = s.read_nodes(0)
    q[5, 0] = 2.0e7  # finite, so the host accepts it
    s.write_nodes(q)
    s.step(1)
    _, boxes = s.observables(raise_unstable=False)
    assert boxes[0]["status_bits"] & P.IBLB_BIT_JUMP, boxes[0]["status_bits"]
    with pytest.raises(P.IblbError) as e:
        s.step(1)
    assert e.value.code == P.IBLB_E_STATE
