"""GPU parity: every stage of the HIP path against the FP64 oracle on the
same seeded inputs, through the C ABI.  Tolerances: FP64 path 1e-10
relative L2 or tighter, FP32 path 1e-5 relative for fields, integer outputs
bit-exact."""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import configs, mesh
from iblb_inputs.configs import Box, Droplet, Workload

from _helpers import deviation, lib_to_oracle_perm, rel_l2, say, to_lib, to_oracle

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3
FULL_U, GRAPH, AUTOTUNE = 4, 1, 2


def sim(wl, storage, flags=0, dev_scale=None):
    import paper_2604_17463_amd as P
    if dev_scale is None:
        dev_scale = 4096.0 if storage == F16 else 1.0
    return P.Simulation(wl, storage=storage, flags=flags, dev_scale=dev_scale)


@pytest.fixture(scope="module")
def perm():
    return lib_to_oracle_perm()


def _empty_box(nx=12, ny=10, nz=8, zbc=0, tau=0.8, g=(1e-5, -2e-5, 3e-5)):
    return Workload("box", [Box(nx, ny, nz, tau=tau, zbc=zbc, body_force=g)], [], storage=F64)


def _perturbed(box, seed, perm):
    _, w, _ = oracle.lattice()
    eta = configs.perturbed_populations(box, seed)
    return (w * box.rho0)[:, None, None, None] * (1.0 + eta)


@pytest.mark.parametrize("storage", [F64, F32, F16, BF16])
def test_rest_state_is_exact(storage):
    say("rest state", storage)
    s = sim(_empty_box(g=(0, 0, 0)), storage, flags=FULL_U)
    s.step(7)
    f, u = s.read_state(0, want_u=True)
    _, w, _ = oracle.lattice()
    c, wl = __import__("paper_2604_17463_amd").velocity_set()
    assert np.array_equal(f, np.broadcast_to(wl[:, None, None, None], f.shape))
    assert np.all(u == 0)
    _, boxes = s.observables()
    assert boxes[0]["mass"] == 12 * 10 * 8 and boxes[0]["max_u"] == 0


@pytest.mark.parametrize("zbc", [0, 1])
@pytest.mark.parametrize("storage", [F64, F32])
def test_lattice_steps_match_oracle(storage, zbc, perm):
    say("lattice steps", storage, zbc)
    wl = _empty_box(zbc=zbc)
    box = wl.boxes[0]
    s = sim(wl, storage, flags=FULL_U)
    s.write_state(to_lib(_perturbed(box, 11, perm), perm))
    f0 = to_oracle(s.read_state(0), perm)  # what the GPU actually holds
    f = f0
    for n in range(1, 6):
        f, _, u = oracle.lb_step(f, box.tau, zbc, None, box.body_force)
        s.step(1)
        fg, ug = s.read_state(0, want_u=True)
        fg = to_oracle(fg, perm)
        # FP64: the oracle stores full f (~w), so its deviations carry
        # ~1e-17/5e-5 = 2e-13 relative rounding of their own
        tol = 2e-12 if storage == F64 else 2e-6
        assert rel_l2(deviation(fg), deviation(f)) < tol * n, n
        assert rel_l2(ug, u) < (1e-12 if storage == F64 else 2e-6), n


# FP32: in the steady state the same rounding of the population update
# (ulp of a deviation ~ 2^-24 of it) recurs every step and is integrated over
# the viscous time H^2/(pi^2 nu) ~ 580 steps; bound ~ (H^2/nu) 2^-24 = 3e-4,
# observed 2.3e-5.  Tolerance 1e-4.
@pytest.mark.parametrize("storage,tol", [(F64, 1e-10), (F32, 1e-4)])
def test_poiseuille_closed_form_gpu(storage, tol):
    say("poiseuille", storage)
    H, tau, g = 24, 0.8, 1e-5
    wl = _empty_box(4, 4, H, 0, tau, (g, 0.0, 0.0))
    s = sim(wl, storage, flags=FULL_U | GRAPH)
    nu = (tau - 0.5) / 3
    s.step(int(36 * H * H / (math.pi ** 2 * nu)))
    _, u = s.read_state(0, want_u=True)
    z = np.arange(H) + 0.5
    lam = (tau - 0.5) ** 2
    exact = g * z * (H - z) / (2 * nu) + (g / nu) * (2 * lam / 3 - 1 / 8)
    ux = u[0, :, 0, 0]
    assert rel_l2(ux, exact) < tol
    assert np.abs(u[0] - u[0, :, :1, :1]).max() <= tol * np.abs(exact).max()


def _c1_jittered(seed=3, amp=0.2):
    wl = configs.plain_c1()
    d = wl.droplets[0]
    d.nodes = configs.jitter_nodes(d.nodes, seed, amp)
    return wl


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("kvol", [0.0, 0.004])
def test_nodal_forces_match_oracle(storage, kvol):
    say("forces", storage, kvol)
    wl = _c1_jittered()
    wl.droplets[0].k_vol = kvol
    s = sim(wl, storage)
    d = wl.droplets[0]
    q0 = d.nodes.copy()
    # move the nodes after init so V differs from V0
    q = configs.jitter_nodes(q0, 8, 0.1)
    s.write_nodes(q)
    qg = s.read_nodes(0)
    A = oracle.wetting_A(d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp)
    want = oracle.node_forces(d.tris, qg, d.sigma, A, d.xi, d.n_exp, d.m_exp, kvol,
                              oracle.volume(d.tris, q0))["phi"]
    got = s.compute_forces(0)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() < (1e-12 if storage == F64 else 2e-5) * scale


@pytest.mark.parametrize("storage", [F64, F32])
def test_bins_and_csr_are_bit_exact(storage):
    say("bins/csr", storage)
    wl = _c1_jittered()
    s = sim(wl, storage)
    q = wl.droplets[0].nodes.copy()
    # put some coordinates exactly on cell faces and centres (ties)
    q[:40, 0] = np.round(q[:40, 0])
    q[40:80, 1] = np.floor(q[40:80, 1]) + 0.5
    q[80:120, 2] = np.floor(q[80:120, 2]) + 0.5
    q[120:130, 0] += 32.0  # unwrapped beyond the box
    s.write_nodes(q)
    qg = s.read_nodes(0)
    assert np.array_equal(oracle.base_cells(qg, 32, 32), s.read_bins(0))
    off, ent = oracle.csr(len(q), wl.droplets[0].tris)
    goff, gent = s.read_csr(0)
    assert np.array_equal(off, goff) and np.array_equal(ent, gent)


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("which", ["c1", "cap", "wrap"])
def test_spread_matches_oracle(storage, which):
    say("spread", storage, which)
    if which == "c1":
        wl = _c1_jittered()
    elif which == "wrap":
        # a droplet across every periodic side of a box whose x and y sizes
        # are not multiples of the band tile (partial last tiles; stencils
        # that wrap touch three tiles along an axis)
        v, t = mesh.sphere(3, 4.0, (36.2, 22.6, 19.1))
        v = configs.jitter_nodes(v, 11, 0.2)
        wl = Workload("wrap", [Box(37, 23, 20, tau=0.9, zbc=1)],
                      [Droplet(0, v, t, sigma=0.01, theta_eq=math.pi, xi=0.4)], storage=F64)
    else:
        v, t = mesh.cap_on_wall(3, 8.0, math.radians(150), 14.5, 17.25, 0.4)
        wl = Workload("cap", [Box(32, 28, 24, tau=0.9)],
                      [Droplet(0, v, t, sigma=0.01, theta_eq=1.0, xi=0.4)], storage=F64)
    s = sim(wl, storage)
    box = wl.boxes[0]
    qg = s.read_nodes(0)
    phi = s.compute_forces(0)
    F, flags = s.compute_spread(0)
    Fo, tw = oracle.spread((box.nz, box.ny, box.nx), box.zbc, qg, phi)
    assert rel_l2(F, Fo) < (1e-13 if storage == F64 else 1e-6)
    tile = __import__("paper_2604_17463_amd").band_tile()
    assert np.array_equal(flags, oracle.touched_tiles(qg, (box.nz, box.ny, box.nx), box.zbc, tile=tile))
    assert np.allclose(F.sum(axis=(1, 2, 3)) + tw, phi.sum(0), rtol=0,
                       atol=(1e-14 if storage == F64 else 1e-7) * np.abs(phi).sum())


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("zbc", [0, 1])
def test_interpolation_matches_oracle(storage, zbc):
    say("interp", storage, zbc)
    wl = _c1_jittered()
    wl.boxes[0].zbc = zbc
    s = sim(wl, storage)
    box = wl.boxes[0]
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3, box.nz, box.ny, box.nx)) * 1e-3
    qg = s.read_nodes(0)
    U = s.interpolate(u, 0)
    Uo = oracle.interp(u, zbc, qg)
    assert rel_l2(U, Uo) < (1e-13 if storage == F64 else 1e-6)


@pytest.mark.parametrize("storage", [F64, F32])
def test_observables_match_oracle_on_same_positions(storage):
    say("observables", storage)
    wl = configs.spreading_c2(steps=1)
    s = sim(wl, storage)
    s.step(3)
    qg = s.read_nodes(0)
    d = wl.droplets[0]
    drops, boxes = s.observables()
    o = oracle.mesh_observables(d.tris, qg, d.xi)
    for k in ("volume", "area", "z_min", "z_max", "height", "contact_radius", "cx", "cy", "cz"):
        assert abs(drops[0][k] - o[k]) <= 1e-11 * max(1.0, abs(o[k])), k
    assert drops[0]["n_crossings"] == o["n_crossings"]
    f = to_oracle(s.read_state(0), lib_to_oracle_perm())
    assert abs(boxes[0]["mass"] - oracle.mass(f)) <= 1e-12 * oracle.mass(f)
    assert abs(boxes[0]["max_u"] - oracle.max_u(f)) <= 1e-9 * max(oracle.max_u(f), 1e-12)


def _run_pair(wl, storage, steps, flags=FULL_U):
    s = sim(wl, storage, flags=flags)
    ref = oracle.OracleSim(wl)
    ref.step(steps)
    s.step(steps)
    return s, ref


def test_plain_c1_fp64_full_parity(perm):
    say("c1 fp64 200 steps")
    wl = configs.plain_c1()
    s, ref = _run_pair(wl, F64, 200)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    assert rel_l2(u, ref.last_u[0]) < 1e-10
    q = s.read_nodes(0)
    assert np.abs(q - ref.q[0]).max() < 1e-10
    drops, boxes = s.observables()
    od, ob = ref.observables()
    assert abs(boxes[0]["mass"] - ob[0]["mass"]) < 1e-13 * ob[0]["mass"]
    for k in ("volume", "area", "height", "contact_radius", "z_min"):
        assert abs(drops[0][k] - od[0][k]) < 1e-10 * abs(od[0][k]), k


def test_plain_c1_fp32_parity(perm):
    say("c1 fp32 200 steps")
    wl = configs.plain_c1()
    s, ref = _run_pair(wl, F32, 200)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(f, ref.f[0]) < 1e-6
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-4
    assert rel_l2(u, ref.last_u[0]) < 1e-5
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-5
    drops, boxes = s.observables()
    od, ob = ref.observables()
    assert abs(boxes[0]["mass"] - ob[0]["mass"]) < 1e-9 * ob[0]["mass"]
    assert abs(drops[0]["volume"] - od[0]["volume"]) < 1e-6 * od[0]["volume"]
    assert abs(drops[0]["height"] - od[0]["height"]) < 1e-5 * od[0]["height"]


def _padded_rows_c1(storage):
    # C1 in a box 30 cells wide: rows padded to 32 cells, little enough that
    # the stream-collide also writes the row padding (zeros) with the row's
    # last line, in every storage
    r = 8.0
    v, t = mesh.sphere(3, r, (15.0, 16.0, 9.0))
    return Workload("padded-rows", [Box(30, 32, 24, tau=1.0)],
                    [Droplet(0, v, t, sigma=0.01, theta_eq=math.radians(90.0), xi=0.05 * r, k_vol=0.0)],
                    storage=storage)


def test_padded_rows_match_oracle(perm):
    say("padded rows fp64 / fp32, 100 steps")
    wl = _padded_rows_c1(F64)
    s, ref = _run_pair(wl, F64, 100)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    assert rel_l2(u, ref.last_u[0]) < 1e-10
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-10
    wl = _padded_rows_c1(F32)
    s, ref = _run_pair(wl, F32, 100)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-4
    assert rel_l2(u, ref.last_u[0]) < 1e-5
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-5


@pytest.mark.parametrize("storage", [F32, F16])
def test_padded_rows_give_identical_results_across_launches(storage):
    say("padded rows, launch shapes", storage)
    wl = _padded_rows_c1(storage)
    ref = None
    for launch in ((32, 2, 1, 0, 0), (64, 1, 1, 1, 0), (64, 2, 2, 0, 3), (128, 2, 1, 1, 0, 1)):
        s = sim(wl, storage, flags=GRAPH)
        s.set_launch(*launch)
        s.step(40)
        got = (s.read_state(0), s.read_nodes(0))
        s.close()
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0]), launch
            assert np.array_equal(got[1], ref[1]), launch


@pytest.mark.parametrize("storage", [F32, F16])
def test_graph_replay_is_bitwise_equal_to_eager(storage):
    say("graph vs eager", storage)
    wl = configs.plain_c1()
    a = sim(wl, storage, flags=0)
    b = sim(wl, storage, flags=GRAPH)
    a.step(37)
    b.step(37)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))


@pytest.mark.parametrize("after", [0, 1])
def test_graphs_of_every_length_match_eager_steps(after):
    # runs of 63, 30, 7 and 2 steps replay the 32-, 16-, 8-, 4- and 2-step
    # graphs and single steps in both schedules; the eager run takes the same
    # 103 steps in one call
    say("graph lengths vs eager, schedule", after)
    wl = configs.plain_c1()
    a = sim(wl, F32, flags=0)
    b = sim(wl, F32, flags=GRAPH)
    for s in (a, b):
        s.set_launch(32, 2, 1, 0, 0, after)
    a.step(103)
    for n in (1, 63, 30, 7, 2):
        b.step(n)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))
    a.close()
    b.close()


def test_runs_are_deterministic():
    say("determinism")
    wl = configs.plain_c1()
    a = sim(wl, F32, flags=GRAPH)
    b = sim(wl, F32, flags=GRAPH | AUTOTUNE)
    a.step(50)
    b.step(50)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))


@pytest.mark.parametrize("storage", [F32, F16])
def test_bulk_launch_configurations_give_identical_results(storage):
    # shape, rows per thread, store policy and grid cap change only the
    # schedule: every cell is computed by the same arithmetic
    say("bulk launch configurations", storage)
    wl = configs.plain_c1()
    ref = None
    for launch in ((32, 2, 1, 0, 0), (64, 1, 2, 0, 0), (64, 4, 2, 1, 0), (64, 2, 1, 1, 5),
                   (64, 1, 2, 0, 3), (256, 1, 2, 1, 1), (32, 2, 1, 0, 0, 1), (64, 1, 2, 1, 7, 1)):
        s = sim(wl, storage, flags=GRAPH)
        s.set_launch(*launch)
        s.step(30)
        got = (s.read_state(0), s.read_nodes(0))
        s.close()
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0]), launch
            assert np.array_equal(got[1], ref[1]), launch


@pytest.mark.parametrize("storage", [F32, F16])
def test_row_segments_give_identical_results(storage):
    # rows longer than threads_x (a multiple of 64) are split into segments
    # that workgroups eight apart take; 20 x 16 = 320 rows leave the last
    # group of eight row groups partly empty for every rows-per-group value
    # below; the 256-wide launch does not segment a 200-cell row
    say("bulk row segments", storage)
    v, t = mesh.sphere_above_wall(2, 4.5, 100.3, 10.2, 0.25)
    wl = Workload("long-rows", [Box(200, 20, 16, tau=0.8)],
                  [Droplet(0, v, t, sigma=0.01, theta_eq=math.radians(70), xi=0.25)], storage=storage)
    ref = None
    for launch in ((256, 1, 1, 0, 0), (64, 1, 1, 0, 0), (64, 2, 2, 1, 0), (128, 1, 2, 0, 3), (64, 4, 1, 1, 7),
                   (128, 2, 1, 0, 0, 1), (64, 1, 1, 1, 8, 1)):
        s = sim(wl, storage, flags=GRAPH)
        s.set_launch(*launch)
        s.step(30)
        got = (s.read_state(0), s.read_nodes(0))
        s.close()
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0]), launch
            assert np.array_equal(got[1], ref[1]), launch


def _small_batch(seed=4):
    rng = np.random.default_rng(seed)
    boxes, drops = [], []
    for k, (nx, ny, nz) in enumerate([(32, 24, 20), (20, 28, 24), (36, 36, 16)]):
        r = float(rng.uniform(4, 6))
        v, t = mesh.sphere_above_wall(2 + k % 2, r, nx / 2 + 0.3, ny / 2 - 0.2, 0.05 * r)
        boxes.append(Box(nx, ny, nz, tau=float(rng.uniform(0.6, 1.4))))
        drops.append(Droplet(k, v, t, sigma=0.01, theta_eq=float(rng.uniform(0.6, 2.5)),
                             xi=0.05 * r, k_vol=0.002 * k))
    return Workload("small-batch", boxes, drops, storage=F32)


@pytest.mark.parametrize("storage", [F64, F32])
def test_batched_boxes_equal_separate_runs(storage):
    say("batched vs separate", storage)
    wl = _small_batch()
    s = sim(wl, storage, flags=GRAPH)
    s.step(25)
    for k in range(len(wl.boxes)):
        one = Workload("one", [wl.boxes[k]], [Droplet(0, **{f: getattr(wl.droplets[k], f) for f in (
            "nodes", "tris", "sigma", "theta_eq", "xi", "n_exp", "m_exp", "k_vol")})],
            storage=storage)
        t = sim(one, storage)
        t.step(25)
        assert np.array_equal(s.read_state(k), t.read_state(0)), k
        assert np.array_equal(s.read_nodes(k), t.read_nodes(0)), k


def test_batched_matches_oracle_fp64(perm):
    say("batched fp64 vs oracle")
    wl = _small_batch()
    s = sim(wl, F64, flags=FULL_U | GRAPH)
    ref = oracle.OracleSim(wl)
    s.step(30)
    ref.step(30)
    for k in range(len(wl.boxes)):
        f = to_oracle(s.read_state(k), perm)
        assert rel_l2(deviation(f), deviation(ref.f[k])) < 1e-10
        assert np.abs(s.read_nodes(k) - ref.q[k]).max() < 1e-10


def test_instability_is_reported_and_sticky():
    import paper_2604_17463_amd as P
    say("instability")
    wl = _empty_box(g=(0.08, 0.0, 0.0), zbc=1)
    s = sim(wl, F32)
    s.step(40)
    with pytest.raises(P.IblbError) as e:
        s.observables()
    assert e.value.code == -5
    with pytest.raises(P.IblbError) as e:
        s.step(1)
    assert e.value.code == -6


def test_set_launch_rejects_shapes_beyond_the_kernel_bound():
    import paper_2604_17463_amd as P
    say("launch shape validation")
    s = sim(configs.plain_c1(), F32)
    for bx, by in ((32, 16), (64, 8), (512, 1), (48, 4)):
        with pytest.raises(P.IblbError) as e:
            s.set_launch(bx, by)
        assert e.value.code == -1
    for bad in ((64, 4, 3, 0, 0), (32, 2, 2, 0, 0), (64, 4, 1, 2, 0), (64, 4, 1, 0, -1),
                (64, 4, 1, 0, 0, 2)):
        with pytest.raises(P.IblbError) as e:
            s.set_launch(*bad)
        assert e.value.code == -1
    s.set_launch(64, 4)
    assert s.get_launch() == (64, 4, 1, 0, 0, 0)
    s.set_launch(64, 4, 2, 1, 7, 1)
    assert s.get_launch() == (64, 4, 2, 1, 7, 1)
    s.step(3)


# ---------------------------------------------------------------- full size
# The 128x128x64 spreading workload (10,242 nodes) in the launch configuration
# the benchmark times (graph replay, autotuned bulk launch shape).

def test_spreading_forces_match_oracle_at_full_size():
    say("spreading forces full size")
    wl = configs.spreading_c2()
    d = wl.droplets[0]
    s = sim(wl, F32, flags=GRAPH | AUTOTUNE)
    s.step(50)
    qg = s.read_nodes(0)
    A = oracle.wetting_A(d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp)
    want = oracle.node_forces(d.tris, qg, d.sigma, A, d.xi, d.n_exp, d.m_exp, d.k_vol,
                              oracle.volume(d.tris, d.nodes))["phi"]
    got = s.compute_forces(0)
    assert np.abs(got - want).max() < 2e-5 * np.abs(want).max()


def test_multidroplet_forces_spread_and_tiles_match_oracle_at_full_size():
    # the 512 x 512 x 256 box with 16 droplets after 20 steps, on the GPU's
    # own node positions: every droplet's nodal forces, the spread force
    # field over all 67 M cells, and the stamped band tiles (bit-exact)
    say("multidroplet full size")
    import paper_2604_17463_amd as P
    wl = configs.multidroplet_c5()
    box = wl.boxes[0]
    shape = (box.nz, box.ny, box.nx)
    s = sim(wl, F32, flags=GRAPH)
    s.step(20)
    Fo, tw, qs, phi_sum, phi_abs = None, np.zeros(3), [], np.zeros(3), 0.0
    for k, d in enumerate(wl.droplets):
        qg = s.read_nodes(k)
        A = oracle.wetting_A(d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp)
        want = oracle.node_forces(d.tris, qg, d.sigma, A, d.xi, d.n_exp, d.m_exp, d.k_vol,
                                  oracle.volume(d.tris, d.nodes))["phi"]
        got = s.compute_forces(k)
        assert np.abs(got - want).max() < 2e-5 * np.abs(want).max(), k
        Fo, t = oracle.spread(shape, box.zbc, qg, got, F=Fo)
        tw += t
        qs.append(qg)
        phi_sum += got.sum(0)
        phi_abs += np.abs(got).sum()
    F, flags = s.compute_spread(0)
    assert rel_l2(F, Fo) < 1e-6
    assert np.array_equal(flags, oracle.touched_tiles(np.concatenate(qs), shape, box.zbc, tile=P.band_tile()))
    assert np.allclose(F.sum(axis=(1, 2, 3)) + tw, phi_sum, rtol=0, atol=1e-7 * phi_abs)
    s.close()


def test_batched_forces_spread_and_tiles_match_oracle_at_full_size():
    # the 64-box batched workload (28 M cells) after 20 steps, on the GPU's
    # own node positions: per droplet its nodal forces, per box the spread
    # force field and the stamped band tiles (bit-exact)
    say("batched full size")
    import paper_2604_17463_amd as P
    wl = configs.batched_c4()
    s = sim(wl, F32, flags=GRAPH)
    s.step(20)
    tile = P.band_tile()
    for k, d in enumerate(wl.droplets):
        box = wl.boxes[d.box]
        shape = (box.nz, box.ny, box.nx)
        qg = s.read_nodes(k)
        A = oracle.wetting_A(d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp)
        want = oracle.node_forces(d.tris, qg, d.sigma, A, d.xi, d.n_exp, d.m_exp, d.k_vol,
                                  oracle.volume(d.tris, d.nodes))["phi"]
        got = s.compute_forces(k)
        assert np.abs(got - want).max() < 2e-5 * np.abs(want).max(), k
        F, flags = s.compute_spread(d.box)
        Fo, tw = oracle.spread(shape, box.zbc, qg, got)
        assert rel_l2(F, Fo) < 1e-6, k
        assert np.array_equal(flags, oracle.touched_tiles(qg, shape, box.zbc, tile=tile)), k
    s.close()


@pytest.mark.parametrize("storage,tol_f", [(F32, 1e-5), (F16, 2.0 ** -11 + 1e-5), (BF16, 2.0 ** -8 + 1e-5)])
def test_spreading_step_matches_oracle_from_gpu_state(storage, tol_f, perm):
    # sampled parity at full size: the oracle advances the GPU's own state
    # (populations and nodes after 200 steps) by one step; the GPU's next
    # step must agree to FP32 rounding, and in FP16 / BF16 deviation storage
    # to the storage rounding of each stored value on top of it
    say("spreading one-step parity full size", storage)
    wl = configs.spreading_c2()
    s = sim(wl, storage, flags=GRAPH | AUTOTUNE)
    s.step(200)
    f0 = to_oracle(s.read_state(0), perm)
    q0 = s.read_nodes(0)
    ref = oracle.OracleSim(wl, f0=[f0])
    ref.q[0] = q0.copy()
    ref.step(1)
    s.step(1)
    f1 = to_oracle(s.read_state(0), perm)
    err_f = rel_l2(deviation(f1), deviation(ref.f[0]))
    say(f"storage {storage}: populations {err_f:.3e}")
    assert err_f < tol_f, err_f
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-6
    drops, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    if storage == F32:
        assert abs(boxes[0]["mass"] - oracle.mass(ref.f[0])) < 1e-9 * oracle.mass(ref.f[0])


# FP16: the oracle starts from the stored state, which it reads exactly; each
# stored deviation of the new state is the FP32 result rounded to FP16,
# within 2^-11 of it relatively, so populations are held to 2^-11 + 1e-5
@pytest.mark.parametrize("storage,tol_f", [(F32, 1e-5), (F16, 5e-4)])
def test_batched_step_matches_oracle_from_gpu_state(storage, tol_f, perm):
    # the 64-box batched workload at full size, autotuned as the bench runs
    # it, after 20 steps: one box in eight (sizes 48 to 128 cells a side, each
    # with its own droplet, contact angle and tau) advanced one step by the
    # oracle from the GPU's own populations and nodes; the GPU's next step of
    # the whole batch must agree in each
    say("batched one-step parity full size", storage)
    wl = configs.batched_c4()
    s = sim(wl, storage, flags=GRAPH | AUTOTUNE)
    s.step(20)
    picks = list(range(0, len(wl.boxes), 8))
    for b in picks:
        assert wl.droplets[b].box == b
    f0 = {b: to_oracle(s.read_state(b), perm) for b in picks}
    q0 = {b: s.read_nodes(b) for b in picks}
    s.step(1)
    drops, boxes = s.observables()
    assert all(bx["status_bits"] == 0 for bx in boxes)
    for b in picks:
        d = wl.droplets[b]
        one = Workload("one", [wl.boxes[b]], [Droplet(0, **{k: getattr(d, k) for k in (
            "nodes", "tris", "sigma", "theta_eq", "xi", "n_exp", "m_exp", "k_vol")})], storage=F64)
        ref = oracle.OracleSim(one, f0=[f0[b]])
        ref.q[0] = q0[b].copy()
        ref.step(1)
        assert ref.below_wall == 0
        f1 = to_oracle(s.read_state(b), perm)
        err_f = rel_l2(deviation(f1), deviation(ref.f[0]))
        err_q = np.abs(s.read_nodes(b) - ref.q[0]).max()
        say(f"box {b} {wl.boxes[b].nx}x{wl.boxes[b].ny}x{wl.boxes[b].nz}: populations {err_f:.3e}, "
            f"nodes {err_q:.3e} lu")
        assert err_f < tol_f, (b, err_f)
        assert err_q < 1e-6, (b, err_q)
    s.close()


# Each storage against the oracle's step from the GPU's own stored state:
# FP64 to its rounding; FP32 to FP32 rounding; FP16 and BF16 deviations to
# their storage rounding of the FP32 result (unit roundoff 2^-11 and 2^-8 of
# each stored value) plus the FP32 bound
@pytest.mark.parametrize("storage,tol_f", [(F64, 1e-10), (F32, 1e-5), (F16, 2.0 ** -11 + 1e-5),
                                           (BF16, 2.0 ** -8 + 1e-5)])
def test_precision_step_matches_oracle_from_gpu_state(storage, tol_f, perm):
    # the 256 x 256 x 128 precision workload (40,962 nodes, tau 0.6),
    # autotuned as the bench runs it, after 50 steps: the oracle advances
    # the GPU's populations and nodes one step; the GPU's next step must
    # agree element by element over the whole box
    say("precision workload one-step parity full size", storage)
    wl = configs.precision_c3(tau=0.6)
    s = sim(wl, storage, flags=GRAPH | AUTOTUNE)
    s.step(50)
    f0 = to_oracle(s.read_state(0), perm)
    q0 = s.read_nodes(0)
    s.step(1)
    drops, boxes = s.observables()
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
    say(f"storage {storage}: populations {err_f:.3e}, nodes {err_q:.3e} lu")
    assert err_f < tol_f, err_f
    assert err_q < (1e-10 if storage == F64 else 1e-6), err_q


@pytest.mark.parametrize("tau_in", [0.0, 1.4])
def test_timing_the_mesh_chain_leaves_the_run_unchanged(tau_in):
    say("mesh chain timing", tau_in)
    wl = configs.plain_c1()
    wl.boxes[0].tau_in = tau_in
    a = sim(wl, F32, flags=GRAPH)
    b = sim(wl, F32, flags=GRAPH)
    a.step(30)
    assert a.time_mesh_chain(reps=5) > 0.0
    a.step(30)
    b.step(60)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))


def test_band_list_longer_than_the_band_grid_equals_separate_runs():
    # nine boxes whose droplets stamp about 34,000 band tiles together, more
    # than the band kernel's 32,768 waves, so that waves take a second tile
    # from the list; alone, each box stamps about 3,800 (one tile per wave).
    # Level-6 meshes (640 node blocks each) keep the node pass in its
    # one-wave form both in the batch and alone (it spreads with four waves,
    # in another summation order, when there are at most as many blocks as
    # compute units).  The batch equals the separate runs bit for bit.
    say("band list longer than the band grid")
    rng = np.random.default_rng(11)
    boxes, drops = [], []
    for k in range(9):
        r = 36.0
        v, t = mesh.sphere_above_wall(6, r, 48.0 + rng.uniform(-2, 2), 48.0 + rng.uniform(-2, 2), 0.05 * r)
        boxes.append(Box(96, 96, 96, tau=float(rng.uniform(0.7, 1.2))))
        drops.append(Droplet(k, v, t, sigma=0.005, theta_eq=float(rng.uniform(0.8, 2.2)), xi=0.05 * r,
                             k_vol=0.0))
    wl = Workload("band-list", boxes, drops, storage=F32)
    s = sim(wl, F32, flags=GRAPH)
    stamped = sum(int(s.compute_spread(b)[1].sum()) for b in range(len(boxes)))
    assert stamped > 32768, stamped
    s.step(10)
    for k in range(len(boxes)):
        one = Workload("one", [boxes[k]], [Droplet(0, **{f: getattr(drops[k], f) for f in (
            "nodes", "tris", "sigma", "theta_eq", "xi", "n_exp", "m_exp", "k_vol")})], storage=F32)
        t = sim(one, F32, flags=GRAPH)
        t.step(10)
        assert np.array_equal(s.read_state(k), t.read_state(0)), k
        assert np.array_equal(s.read_nodes(k), t.read_nodes(0)), k
        t.close()
    s.close()


@pytest.mark.parametrize("storage", [F32, F16])
def test_batch_with_boxes_without_droplets_equals_separate_runs(storage):
    # boxes 0 and 2 hold no droplet (body-force channels, one z-periodic);
    # box 1 the C1 droplet: each equals its own run bit for bit
    say("batch with empty boxes", storage)
    c1 = configs.plain_c1()
    e0 = Box(20, 12, 16, tau=0.7, body_force=(2e-5, 0.0, 0.0))
    e2 = Box(36, 8, 10, tau=1.2, zbc=1, body_force=(0.0, 1e-5, -1e-5))
    d = c1.droplets[0]
    d.box = 1
    wl = Workload("mixed", [e0, c1.boxes[0], e2], [d], storage=storage)
    s = sim(wl, storage, flags=GRAPH)
    s.step(30)
    singles = [Workload("e0", [e0], [], storage=storage), configs.plain_c1(),
               Workload("e2", [e2], [], storage=storage)]
    for k, one in enumerate(singles):
        t = sim(one, storage, flags=GRAPH)
        t.step(30)
        assert np.array_equal(s.read_state(k), t.read_state(0)), k
    t = sim(singles[1], storage, flags=GRAPH)
    t.step(30)
    assert np.array_equal(s.read_nodes(0), t.read_nodes(0))
