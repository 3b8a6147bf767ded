"""Pins of the oracle's interface forces and mesh geometry (paper Sec. 2,
Eqs. 9-11) against closed forms, exact identities and finite differences.
CPU only."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from iblb_inputs import mesh

RNG = np.random.default_rng(7)


def _cube():
    v = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=float)
    # two triangles per face, counter-clockwise seen from outside
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return v, np.array(t, dtype=np.int32)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_icosphere_counts_and_orientation(level):
    v, t = mesh.icosphere(level)
    assert len(v) == 10 * 4 ** level + 2 and len(t) == 20 * 4 ** level
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    assert mesh.is_closed_oriented(t)
    assert oracle.volume(t, v) > 0


def test_cube_volume_and_area_exact():
    v, t = _cube()
    assert mesh.is_closed_oriented(t)
    assert abs(oracle.volume(t, v) - 1.0) < 1e-15
    assert abs(oracle.area(t, v) - 6.0) < 1e-14
    # translation invariance of the closed-mesh volume formula
    assert abs(oracle.volume(t, v + [3.0, -7.0, 11.0]) - 1.0) < 1e-13
    A, n = oracle.triangle_geometry(t, v)
    assert np.allclose(A, 0.5)
    assert np.allclose(np.abs(n).sum(1), 1.0)


def test_sphere_volume_area_converge():
    v, t = mesh.icosphere(6)
    assert abs(oracle.area(t, v) - 4 * math.pi) / (4 * math.pi) < 1e-3
    assert abs(oracle.volume(t, v) - 4 * math.pi / 3) / (4 * math.pi / 3) < 1e-3


def test_paper_sec4_workloads_follow_the_paper():
    # the two wetting runs of Sec. 4 (tests/golden/paper_spreading_sec4.txt)
    import os
    from iblb_inputs import configs
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_spreading_sec4.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            g[k] = [float(x) for x in v]
    r0 = g["R0"][0]
    wls = {"CAP": configs.paper_cap45(), "NECK": configs.paper_neck()}
    for key, wl in wls.items():
        b, d = wl.boxes[0], wl.droplets[0]
        assert (b.nx, b.ny, b.nz) == tuple(int(x) for x in g[key + "_LATTICE"])
        assert abs(b.tau - g[key + "_TAU"][0]) < 1e-12
        assert abs(math.degrees(d.theta_eq) - g["THETA_EQ_DEG"][0]) < 1e-9
        assert d.sigma == g["SIGMA"][0] and abs(d.xi - g["XI_OVER_R0"][0] * r0) < 1e-12
        assert abs(len(d.tris) / g["TRIANGLES"][0] - 1.0) < 0.02
        assert mesh.is_closed_oriented(d.tris)
        # the volume of the sphere of radius R0 (mesh error of the 59,292 nodes)
        assert abs(oracle.volume(d.tris, d.nodes) / (4 * math.pi * r0 ** 3 / 3) - 1.0) < 2e-3
        assert abs(d.nodes[:, 2].min() - d.xi) < 1e-9
    # the cap starts at 90 deg, the sphere as a sphere of radius R0
    cap, neck = wls["CAP"].droplets[0].nodes, wls["NECK"].droplets[0].nodes
    assert abs(cap[:, 2].max() - cap[:, 2].min() - mesh.cap_radius(r0, math.pi / 2)) < 0.05
    c = neck.mean(axis=0)
    assert np.abs(np.linalg.norm(neck - c, axis=1) / r0 - 1.0).max() < 1e-9


def _jittered(level=1, r=2.0, amp=0.1, centre=(5.0, 6.0, 7.0)):
    v, t = mesh.sphere(level, r, centre)
    return v + RNG.uniform(-amp, amp, v.shape), t


def test_surface_tension_is_minus_sigma_area_gradient():
    v, t = _jittered()
    sigma = 0.37
    out = oracle.node_forces(t, v, sigma, 0.0, 1.0)
    h = 1e-6
    fd = np.zeros_like(v)
    for j in range(len(v)):
        for a in range(3):
            vp, vm = v.copy(), v.copy()
            vp[j, a] += h
            vm[j, a] -= h
            fd[j, a] = -sigma * (oracle.area(t, vp) - oracle.area(t, vm)) / (2 * h)
    assert np.allclose(out["phi_st"], fd, rtol=0, atol=1e-8)


def test_surface_tension_identities():
    v, t = _jittered(level=3, r=8.0, amp=0.3)
    sigma = 0.01
    st = oracle.node_forces(t, v, sigma, 0.0, 1.0)["phi_st"]
    A = oracle.area(t, v)
    assert np.abs(st.sum(0)).max() < 1e-15
    assert np.abs(np.cross(v, st).sum(0)).max() < 1e-13
    # area is homogeneous of degree 2 about any origin
    c = v.mean(0)
    assert abs(np.sum((v - c) * st) + 2 * sigma * A) < 1e-12


def test_surface_tension_on_sphere_is_laplace_pressure():
    r = 8.0
    v, t = mesh.sphere(5, r, (0.0, 0.0, 0.0))
    sigma = 0.01
    out = oracle.node_forces(t, v, sigma, 0.0, 1.0)
    # exact: sum_j n_j.phi_j = -2 sigma A / R for a sphere centred at 0 (nodes on it)
    A = oracle.area(t, v)
    assert abs(np.sum(v / r * out["phi_st"]) + 2 * sigma * A / r) < 1e-12
    # per node, the force is close to the Laplace pressure times the node's
    # area share (the 12 valence-5 vertices deviate most)
    lap = -2 * sigma / r * (out["chi"] / 3)[:, None] * v / r
    rel = np.linalg.norm(out["phi_st"] - lap, axis=1) / np.linalg.norm(lap, axis=1)
    assert np.median(rel) < 0.02 and rel.max() < 0.2


def test_volume_penalty_gradient():
    v, t = _jittered()
    k, V0 = 0.5, 20.0
    out = oracle.node_forces(t, v, 0.0, 0.0, 1.0, k_vol=k, V0=V0)
    V = oracle.volume(t, v)
    grad = out["phi_v"] / (-k * (V - V0) / V0)
    h = 1e-6
    fd = np.zeros_like(v)
    for j in range(len(v)):
        for a in range(3):
            vp, vm = v.copy(), v.copy()
            vp[j, a] += h
            vm[j, a] -= h
            fd[j, a] = (oracle.volume(t, vp) - oracle.volume(t, vm)) / (2 * h)
    assert np.allclose(grad, fd, rtol=0, atol=1e-7)
    assert abs(np.sum((v - v.mean(0)) * grad) - 3 * V) < 1e-10
    assert np.all(oracle.node_forces(t, v, 0.0, 0.0, 1.0, k_vol=0.0, V0=V0)["phi_v"] == 0)


@pytest.mark.parametrize("nm", [(9, 3), (4, 3), (3, 2), (12, 6)])
@pytest.mark.parametrize("theta_deg", [30.0, 60.0, 90.0, 150.0])
def test_wetting_amplitude_integral_identity(nm, theta_deg):
    # Eq. 11 is the choice of A for which the work of the interaction from
    # the film to infinity balances the spreading coefficient:
    #   int_xi^inf Pi(d) dd = -sigma (1 + cos theta_eq).
    n, m = nm
    sigma, xi = 0.005, 1.2
    th = math.radians(theta_deg)
    A = oracle.wetting_A(sigma, th, xi, n, m)
    val, err = quad(lambda d: oracle.pi_of_d(d, A, xi, n, m), xi, np.inf, epsabs=1e-14,
                    epsrel=1e-12, limit=400)
    assert abs(val + sigma * (1 + math.cos(th))) < 1e-9 * sigma
    assert abs(oracle.pi_of_d(xi, A, xi, n, m)) < 1e-18
    assert oracle.pi_of_d(0.9 * xi, A, xi, n, m) > 0 > oracle.pi_of_d(1.5 * xi, A, xi, n, m)


def test_wetting_amplitude_special_cases():
    assert oracle.wetting_A(0.01, math.pi, 0.4) == pytest.approx(0.0, abs=1e-18)
    # (9,3): A = sigma * 2*8/(6 xi) (1 + cos theta)
    assert oracle.wetting_A(0.01, math.pi / 2, 0.4) == pytest.approx(0.01 * 16 / 6 / 0.4, rel=1e-15)


def test_wetting_force_on_flat_bottom_patch():
    # Cap mesh: nodes strictly inside the flat disc have only flat, downward
    # neighbours, so n_j = -z and phi_Pi,j = +chi_j Pi(d) / 3 z exactly.
    xi = 1.2
    v, t = mesh.cap_on_wall(3, 8.0, math.radians(150.0), 0.0, 0.0, xi)
    sigma, th = 0.005, math.radians(60.0)
    A = oracle.wetting_A(sigma, th, xi)
    out = oracle.node_forces(t, v, sigma, A, xi)
    flat = np.zeros(len(v), bool)
    on = np.abs(v[:, 2] - xi) < 1e-12
    for j in np.nonzero(on)[0]:
        ring = t[(t == j).any(1)]
        flat[j] = np.all(on[ring])
    assert flat.sum() >= 3
    Pi = oracle.pi_of_d(xi, A, xi)
    for j in np.nonzero(flat)[0]:
        assert np.allclose(out["nhat"][j], [0, 0, -1], atol=1e-15)
        assert np.allclose(out["phi_pi"][j], [0, 0, out["chi"][j] * Pi / 3], atol=1e-18)
    # one-third shares of the 1-ring areas add up to the total area
    assert abs(out["chi"].sum() / 3 - oracle.area(t, v)) < 1e-11
    # attraction toward the wall for a patch above xi
    v2 = v.copy()
    v2[:, 2] += 0.5
    out2 = oracle.node_forces(t, v2, sigma, A, xi)
    assert np.all(out2["phi_pi"][flat, 2] < 0)


def test_below_wall_nodes_are_counted():
    v, t = mesh.sphere(2, 3.0, (5.0, 5.0, 2.0))
    out = oracle.node_forces(t, v, 0.01, 0.1, 0.2)
    assert out["below_wall"] == int(np.sum(v[:, 2] <= 0))
    assert out["below_wall"] > 0


def test_csr_brute_force():
    v, t = mesh.icosphere(3)
    off, ent = oracle.csr(len(v), t)
    for j in range(len(v)):
        want = sorted(3 * ti + c for ti in range(len(t)) for c in range(3) if t[ti, c] == j)
        assert list(ent[off[j]:off[j + 1]]) == want


def test_mesh_observables_on_a_cap():
    # Cap of angle theta0 on the plane z = xi, from a sphere of radius Rc
    # centred at height xi - Rc cos(theta0): the plane z_c = z_min + xi cuts
    # it in a circle of radius sqrt(Rc^2 - (2 xi - zc)^2).
    R, xi, th0 = 24.0, 1.2, math.radians(150.0)
    v, t = mesh.cap_on_wall(6, R, th0, 64.0, 64.0, xi)
    o = oracle.mesh_observables(t, v, xi)
    rc = mesh.cap_radius(R, th0)
    zc = xi - rc * math.cos(th0)
    assert abs(o["z_min"] - xi) < 1e-12
    assert abs(o["height"] - (zc + rc - xi)) < 1e-3 * rc
    want_r = math.sqrt(rc ** 2 - (2 * xi - zc) ** 2)
    assert abs(o["contact_radius"] - want_r) < 2e-3 * want_r
    assert abs(o["cx"] - 64.0) < 1e-9 and abs(o["cy"] - 64.0) < 1e-9
    assert abs(o["volume"] - 4 / 3 * math.pi * R ** 3) / (4 / 3 * math.pi * R ** 3) < 5e-3
    assert o["theta_app"] == pytest.approx(2 * math.atan(o["height"] / o["contact_radius"]))
