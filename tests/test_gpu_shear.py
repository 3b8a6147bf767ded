"""GPU parity of the moving walls and the deformation index (paper Sec. 4:
a free droplet in the shear flow between two moving walls) against the FP64
oracle, through the C ABI, and the closed forms they must reach.

Tolerances as for resting walls: lattice steps 2e-12 n (FP64) and 2e-6 n
(FP32) relative L2 of the deviations; whole steps 1e-10 (FP64); Couette
flow within 1e-10 U (FP64) and 1e-4 U (FP32 storage of deviations of size
~U); the deformation index within 1e-10 of the oracle's on the same
positions."""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import configs, mesh
from iblb_inputs.configs import Box, Droplet, Workload

from _helpers import deviation, lib_to_oracle_perm, rel_l2, say, to_lib, to_oracle

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1
FULL_U, GRAPH = 4, 1


def sim(wl, storage, flags=0):
    import paper_2604_17463_amd as P
    return P.Simulation(wl, storage=storage, flags=flags, dev_scale=1.0)


@pytest.fixture(scope="module")
def perm():
    return lib_to_oracle_perm()


def couette_populations(box, gamma):
    """Equilibrium populations of u = (gamma (z + 1/2 - nz/2), 0, 0), rho = 1
    (the oracle's f^eq), oracle order."""
    f = np.empty((19, box.nz, box.ny, box.nx))
    feq = np.zeros(19)
    for k in range(box.nz):
        oracle.lib().orc_feq(1.0, np.array([gamma * (k + 0.5 - box.nz / 2.0), 0.0, 0.0]), feq)
        f[:, k] = feq[:, None, None]
    return f


@pytest.mark.parametrize("storage", [F64, F32])
def test_moving_wall_lattice_steps_match_oracle(storage, perm):
    say("moving wall lattice steps", storage)
    box = Box(10, 8, 12, tau=0.7, body_force=(1e-5, 0.0, -2e-5), wall_lo=(0.02, -0.01),
              wall_hi=(-0.03, 0.015))
    wl = Workload("walls", [box], [], storage=storage)
    s = sim(wl, storage, flags=FULL_U)
    _, w, _ = oracle.lattice()
    f = (w * box.rho0)[:, None, None, None] * (1.0 + configs.perturbed_populations(box, 21))
    s.write_state(to_lib(f, perm))
    f = to_oracle(s.read_state(0), perm)
    uw = (box.wall_lo, box.wall_hi)
    for n in range(1, 6):
        f, _, u = oracle.lb_step(f, box.tau, 0, None, box.body_force, u_wall=uw, rho_wall=box.rho0)
        s.step(1)
        fg, ug = s.read_state(0, want_u=True)
        fg = to_oracle(fg, perm)
        tol = 2e-12 if storage == F64 else 2e-6
        assert rel_l2(deviation(fg), deviation(f)) < tol * n, n
        assert rel_l2(ug, u) < (1e-12 if storage == F64 else 2e-6), n


@pytest.mark.parametrize("storage,tol", [(F64, 1e-10), (F32, 1e-4)])
def test_couette_flow_closed_form_gpu(storage, tol):
    say("couette", storage)
    H, U = 16, 0.01
    wl = Workload("couette", [Box(4, 4, H, tau=0.8, wall_lo=(-U, 0.0), wall_hi=(U, 0.0))], [],
                  storage=storage)
    s = sim(wl, storage, flags=FULL_U | GRAPH)
    s.step(40000)
    _, u = s.read_state(0, want_u=True)
    z = np.arange(H) + 0.5
    exact = U * (2 * z / H - 1)
    assert np.abs(u[0, :, 0, 0] - exact).max() < tol * U
    assert np.abs(u[0] - u[0, :, :1, :1]).max() < tol * U
    _, boxes = s.observables()
    assert abs(boxes[0]["mass"] - 4 * 4 * H) < (1e-12 if storage == F64 else 1e-6) * 4 * 4 * H


def _rot_y(v, phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.stack([c * v[:, 0] - s * v[:, 2], v[:, 1], s * v[:, 0] + c * v[:, 2]], axis=1)


@pytest.mark.parametrize("storage", [F64, F32])
def test_deformation_index_matches_oracle(storage):
    say("deformation observable", storage)
    v, t = mesh.sphere(4, 6.0, (0.0, 0.0, 0.0))
    v = _rot_y(v * np.array([1.3, 1.0, 0.75]), 0.5) + np.array([16.0, 12.0, 14.0])
    d = Droplet(0, v, t, sigma=0.01, theta_eq=math.pi, xi=0.3, k_vol=0.0)
    wl = Workload("ellipsoid", [Box(32, 24, 28, tau=0.9)], [d], storage=storage)
    s = sim(wl, storage)
    for steps in (0, 3):
        s.step(steps)
        got = s.observables()[0][0]
        want = oracle.deformation(t, s.read_nodes(0))
        assert abs(got["deformation"] - want["D"]) < 1e-10
        assert abs(got["inclination"] - want["inclination"]) < 1e-10
    # the starting shape itself: D = (a - c) / (a + c), inclination 0.5
    s2 = sim(wl, storage)
    o = s2.observables()[0][0]
    assert abs(o["deformation"] - 0.55 / 2.05) < 1e-6
    assert abs(o["inclination"] - 0.5) < 1e-6


@pytest.mark.parametrize("lam", [1.0, 3.0])
def test_shear_droplet_fp64_parity(lam, perm):
    say("shear droplet fp64 parity", lam)
    wl = configs.shear_droplet(lam=lam, r=6.0, ca=0.2, re=0.5, shape=(32, 24, 32), level=3,
                               storage=F64)
    f0 = couette_populations(wl.boxes[0], wl.extra["shear_rate"])
    s = sim(wl, F64, flags=FULL_U)
    s.write_state(to_lib(f0, perm))
    ref = oracle.OracleSim(wl, f0=[to_oracle(s.read_state(0), perm)])
    ref.step(200)
    s.step(200)
    f, u = s.read_state(0, want_u=True)
    f = to_oracle(f, perm)
    assert rel_l2(deviation(f), deviation(ref.f[0])) < 1e-10
    assert rel_l2(u, ref.last_u[0]) < 1e-10
    assert np.abs(s.read_nodes(0) - ref.q[0]).max() < 1e-10
    got = s.observables()[0][0]
    want = ref.observables()[0][0]
    assert abs(got["deformation"] - want["deformation"]) < 1e-9
    assert got["deformation"] > 1e-3  # the shear has deformed it


@pytest.mark.parametrize("lam", [1.0, 3.0])
def test_free_droplet_in_shear_reaches_taylor_deformation(lam, perm):
    # Sec. 4: in the Stokes limit at small Ca the deformation index tends to
    # D_inf = (19 lam + 16) / (16 lam + 16) Ca (Eq. D_inf); the paper's own
    # run is 2.7 % off at lam = 1.  Here R = 12, Ca = 0.05, Re = 0.01 in a
    # 128 x 96 x 192 channel (walls 8 R from the centre, which adds about 2 % of
    # confinement), 16 capillary times mu_out R / sigma from a Couette flow.
    # Measured: D / D_inf = 1.034 (lam = 1), 0.994 (lam = 3); 5 % allowed.
    say("taylor deformation", lam)
    wl = configs.shear_droplet(lam=lam)
    s = sim(wl, F32, flags=GRAPH)
    s.write_state(to_lib(couette_populations(wl.boxes[0], wl.extra["shear_rate"]), perm))
    dinf = (19 * lam + 16) / (16 * lam + 16) * wl.extra["ca"]
    tc = wl.extra["t_cap"]
    d0 = s.observables()[0][0]
    history = []
    for k in range(1, 9):
        s.step(int(round(2 * tc)))
        d, b = s.observables()
        history.append(d[0]["deformation"])
    assert abs(history[-1] / dinf - 1.0) < 0.05, history[-1] / dinf
    assert all(b > a for a, b in zip(history[:5], history[1:6]))   # monotone approach
    # the approach: first-order small-deformation relaxation toward the
    # final value, D(t) = D_end (1 - exp(-t / t_d)) with
    # t_d = (19 lam + 16)(2 lam + 3) / (40 (lam + 1)) mu_out R / sigma
    # (measured within 0.003 at lam = 1 and 0.025 at lam = 3)
    t_d = (19 * lam + 16) * (2 * lam + 3) / (40 * (lam + 1))
    for k, t in enumerate((2.0, 4.0, 6.0)):
        assert abs(history[k] / history[-1] - (1 - math.exp(-t / t_d))) < 0.04, (t, history[k])
    assert 35.0 < math.degrees(d[0]["inclination"]) < 45.0
    assert abs(d[0]["volume"] / d0["volume"] - 1.0) < 0.005
    assert abs(d[0]["cz"] - wl.boxes[0].nz / 2.0) < 1e-3        # stays on the centre plane


def test_moving_walls_graph_replay_is_bitwise_equal_to_eager():
    # 37 steps: one single-step graph, one 32-step graph, four single steps
    say("moving walls graph vs eager")
    wl = configs.shear_droplet(lam=2.0, r=6.0, ca=0.2, re=0.5, shape=(32, 24, 32), level=3,
                               storage=F32)
    a = sim(wl, F32, flags=0)
    b = sim(wl, F32, flags=GRAPH)
    a.step(37)
    b.step(37)
    assert np.array_equal(a.read_state(0), b.read_state(0))
    assert np.array_equal(a.read_nodes(0), b.read_nodes(0))
    assert a.observables()[0][0]["deformation"] == b.observables()[0][0]["deformation"]


def test_shear_step_at_paper_size_matches_oracle_from_gpu_state(perm):
    # both options at the scale of the paper's shear run (204 x 152 x 304,
    # r = 19, 10,242 nodes), with a viscosity ratio of 3 (tau_in 2.0, tau
    # 1.0) and both walls moving: after 50 steps (graphs, autotuned launch),
    # the inside bits equal the oracle's at the GPU's node positions (exact),
    # and the oracle's step from the GPU's populations and nodes matches the
    # GPU's next step (deviations 1e-5 relative L2, nodes 1e-6 lu)
    say("shear droplet at paper size, lambda 3: one step against the oracle")
    autotune = 2
    wl = configs.shear_droplet(lam=3.0, r=19.0, shape=(204, 152, 304), level=5)
    box = wl.boxes[0]
    s = sim(wl, F32, flags=GRAPH | autotune)
    s.step(50)
    f0 = to_oracle(s.read_state(0), perm)
    q0 = s.read_nodes(0)
    inside = s.read_inside(0)
    want = oracle.inside((box.nz, box.ny, box.nx), np.asarray(wl.droplets[0].tris, np.int32), q0)
    assert np.array_equal(inside, want)
    assert 0 < int(inside.sum()) < inside.size
    s.step(1)
    drops, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    f1 = to_oracle(s.read_state(0), perm)
    q1 = s.read_nodes(0)
    s.close()
    ref = oracle.OracleSim(wl, f0=[f0])
    ref.q[0] = q0.copy()
    ref.step(1)
    err_f = rel_l2(deviation(f1), deviation(ref.f[0]))
    err_q = np.abs(q1 - ref.q[0]).max()
    say(f"populations {err_f:.3e}, nodes {err_q:.3e} lu, inside cells {int(inside.sum())}")
    assert err_f < 1e-5, err_f
    assert err_q < 1e-6, err_q
