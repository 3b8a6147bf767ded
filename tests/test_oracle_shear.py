"""Pins of the oracle's moving walls and deformation index (paper Sec. 4:
a free droplet between two walls driving a shear flow, deformation index
D = (r1 - r3) / (r1 + r3) from the semi-axes in the shear plane).  CPU only.

Moving walls: plane Couette flow is an exact steady state of BGK with
halfway bounce-back, and a fluid moving with both walls stays at rest
relative to them.  Deformation index: the affine image A P of a polyhedron
P with isotropic second moments k I has second moments k A A^T, so a
scaled and rotated icosphere (isotropic by icosahedral symmetry) or a
rotated cuboid has D = (a - c) / (a + c) and inclination phi exactly."""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import mesh

C, W, _ = oracle.lattice()


def test_couette_flow_between_moving_walls_is_linear():
    H, n, U = 16, 4, 0.01
    f = np.broadcast_to(W[:, None, None, None], (19, H, n, n)).copy()
    for _ in range(40000):
        f, rho, u = oracle.lb_step(f, 0.8, 0, None, (0, 0, 0), u_wall=((-U, 0.0), (U, 0.0)))
    z = np.arange(H) + 0.5
    exact = U * (2 * z / H - 1)
    assert np.abs(u[0, :, 0, 0] - exact).max() < 1e-11 * U
    assert np.abs(u[1]).max() == 0.0 and np.abs(u[2]).max() < 1e-14
    assert abs(oracle.mass(f) - H * n * n) < 1e-12 * H * n * n


@pytest.mark.parametrize("uw", [(0.02, -0.01), (-0.03, 0.0)])
def test_fluid_moving_with_both_walls_is_steady(uw):
    # the equilibrium at u = (uw, 0) is a fixed point only if the wall term
    # has the right sign and size in every reflected direction
    feq = np.zeros(19)
    oracle.lib().orc_feq(1.0, np.array([uw[0], uw[1], 0.0]), feq)
    f = np.broadcast_to(feq[:, None, None, None], (19, 6, 5, 4)).copy()
    g, _, u = oracle.lb_step(f, 0.9, 0, None, (0, 0, 0), u_wall=(uw, uw))
    assert np.abs(g - f).max() < 1e-16
    # resting walls do not keep it
    g0, _, _ = oracle.lb_step(f, 0.9, 0, None, (0, 0, 0))
    assert np.abs(g0 - f).max() > 1e-4


def test_moving_walls_conserve_mass():
    rng = np.random.default_rng(7)
    f = W[:, None, None, None] * (1 + 1e-2 * rng.standard_normal((19, 8, 6, 5)))
    m0 = oracle.mass(f)
    for _ in range(20):
        f, _, _ = oracle.lb_step(f, 0.7, 0, None, (1e-5, 0, 0), u_wall=((0.03, -0.02), (-0.01, 0.04)))
    assert abs(oracle.mass(f) - m0) < 1e-13 * m0


def _rot_y(v, phi):
    # rotation in the x-z plane taking the x axis toward +z by phi
    c, s = math.cos(phi), math.sin(phi)
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    return np.stack([c * x - s * z, y, s * x + c * z], axis=1)


def _cuboid(a, b, c):
    v = np.array([[sx * a, sy * b, sz * c] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                 dtype=float)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for p, q, r, s in quads:
        t += [(p, q, r), (p, r, s)]
    return v, np.array(t, dtype=np.int32)


def test_volume_moments_of_a_cuboid():
    a, b, c = 3.0, 2.0, 1.5
    v, t = _cuboid(a, b, c)
    ref = np.array([0.7, -1.1, 0.4])
    V, M1, M2 = oracle.volume_moments(t, v + 5.0, ref)
    assert abs(V - 8 * a * b * c) < 1e-12
    assert np.allclose(M1, V * (5.0 - ref), rtol=1e-13, atol=1e-12)
    # about the centre: diag(V a^2/3, V b^2/3, V c^2/3)
    Vc, M1c, M2c = oracle.volume_moments(t, v, np.zeros(3))
    assert np.allclose(M2c, np.diag([Vc * a * a / 3, Vc * b * b / 3, Vc * c * c / 3]), atol=1e-12)


@pytest.mark.parametrize("phi", [0.0, 0.3, -0.7, math.pi / 4])
def test_deformation_of_a_rotated_cuboid(phi):
    a, b, c = 4.0, 2.5, 2.0
    v, t = _cuboid(a, b, c)
    v = _rot_y(v, phi) + np.array([10.0, 11.0, 12.0])
    d = oracle.deformation(t, v)
    assert abs(d["D"] - (a - c) / (a + c)) < 1e-12
    assert abs(d["inclination"] - phi) < 1e-12
    assert abs(d["r1"] - a * math.sqrt(5 / 3)) < 1e-12
    assert np.allclose(d["centroid"], [10.0, 11.0, 12.0], atol=1e-12)


@pytest.mark.parametrize("level", [2, 4])
def test_deformation_of_a_sphere_mesh_is_zero(level):
    v, t = mesh.sphere(level, 7.0, (20.0, 20.0, 20.0))
    assert oracle.deformation(t, v)["D"] < 1e-12


@pytest.mark.parametrize("phi", [0.0, 0.4, 1.2])
def test_deformation_of_an_affine_icosphere(phi):
    a, b, c = 1.25, 1.0, 0.8
    v, t = mesh.sphere(4, 9.0, (0.0, 0.0, 0.0))
    v = _rot_y(v * np.array([a, b, c]), phi) + np.array([30.0, 20.0, 25.0])
    d = oracle.deformation(t, v)
    assert abs(d["D"] - (a - c) / (a + c)) < 1e-12
    assert abs(d["inclination"] - phi) < 1e-12
