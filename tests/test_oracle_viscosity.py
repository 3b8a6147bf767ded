"""Pins of the oracle's viscosity contrast (paper Sec. 2, below Eq. 13: fluid
nodes inside the droplet relax with tau_in, found by ray tracing).  CPU only.

The inside test is checked on meshes whose interior is known exactly (boxes,
spheres, two meshes, a droplet across the periodic boundary) including the
tie rule; the per-cell relaxation time on a layered channel flow whose
steady profile is known in closed form away from the viscosity jump."""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import mesh

C, W, _ = oracle.lattice()


def _box_mesh(lo, hi):
    v = np.array([[(lo[0], hi[0])[x], (lo[1], hi[1])[y], (lo[2], hi[2])[z]]
                  for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=float)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    t = np.array(t, dtype=np.int32)
    assert mesh.is_closed_oriented(t) and oracle.volume(t, v) > 0
    return v, t


def _centres(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 for n in (nz, ny, nx)], indexing="ij")
    return x, y, z


def test_inside_of_a_box_is_its_interior():
    shape = (6, 8, 10)
    lo, hi = (2.3, 1.2, 0.7), (7.6, 5.9, 4.4)
    v, t = _box_mesh(lo, hi)
    x, y, z = _centres(shape)
    want = (x > lo[0]) & (x < hi[0]) & (y > lo[1]) & (y < hi[1]) & (z > lo[2]) & (z < hi[2])
    assert np.array_equal(oracle.inside(shape, t, v), want.astype(np.uint8))


def test_inside_ties_follow_the_perturbation_rule():
    # faces on cell-centre planes: the column point moves by (+eps, +eps^2),
    # so x = lo and y = lo are inside, x = hi and y = hi outside; a crossing
    # at the height of a centre counts as below it, so z = lo is inside and
    # z = hi outside.  The interior is [lo, hi) on every axis.
    shape = (10, 10, 10)
    v, t = _box_mesh((2.5, 2.5, 2.5), (6.5, 6.5, 6.5))
    x, y, z = _centres(shape)
    want = (x >= 2.5) & (x < 6.5) & (y >= 2.5) & (y < 6.5) & (z >= 2.5) & (z < 6.5)
    got = oracle.inside(shape, t, v)
    assert got.sum() == 64
    assert np.array_equal(got, want.astype(np.uint8))


def test_inside_of_a_sphere_mesh():
    # the icosphere's faces lie inside the sphere and outside 0.95 R
    shape = (18, 20, 20)
    c, R = np.array([10.3, 9.7, 8.2]), 6.0
    v, t = mesh.sphere(3, R, c)
    x, y, z = _centres(shape)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    got = oracle.inside(shape, t, v)
    assert np.all(got[r < 0.95 * R] == 1)
    assert np.all(got[r > R] == 0)
    # cell count against the mesh volume: one cell per unit volume
    assert abs(got.sum() - oracle.volume(t, v)) < 0.03 * oracle.volume(t, v)


def test_inside_over_two_meshes_and_across_the_periodic_side():
    shape = (16, 24, 32)
    nz, ny, nx = shape
    (v1, t1) = mesh.sphere(3, 5.0, (31.0, 12.0, 8.0))      # straddles x = nx (unwrapped)
    (v2, t2) = mesh.sphere(3, 4.0, (14.0, 11.5, 7.5))
    v = np.concatenate([v1, v2])
    t = np.concatenate([t1, t2 + len(v1)])
    x, y, z = _centres(shape)
    dx = (x - 31.0 + nx / 2) % nx - nx / 2
    r1 = np.sqrt(dx ** 2 + (y - 12.0) ** 2 + (z - 8.0) ** 2)
    r2 = np.sqrt((x - 14.0) ** 2 + (y - 11.5) ** 2 + (z - 7.5) ** 2)
    got = oracle.inside(shape, t, v)
    assert np.all(got[(r1 < 0.95 * 5.0) | (r2 < 0.95 * 4.0)] == 1)
    assert np.all(got[(r1 > 5.0) & (r2 > 4.0)] == 0)
    # both images of the straddling sphere are found: cells at x < 4 and x > 28
    assert got[:, :, :4].sum() > 0 and got[:, :, 28:].sum() > 0


def test_tau_in_equal_to_tau_changes_nothing():
    rng = np.random.default_rng(5)
    f = W[:, None, None, None] * (1 + 1e-3 * rng.standard_normal((19, 6, 5, 4)))
    mask = (rng.random((6, 5, 4)) < 0.5).astype(np.uint8)
    a, _, _ = oracle.lb_step(f, 0.8, 0, None, (1e-5, 0, 0))
    b, _, _ = oracle.lb_step(f, 0.8, 0, None, (1e-5, 0, 0), inside=mask, tau_in=0.8)
    assert np.array_equal(a, b)


def test_layered_channel_flow_with_two_viscosities():
    # Body-force driven flow between halfway bounce-back walls (z = 0, H) with
    # a central layer of relaxation time tau_in.  The shear stress is fixed by
    # the force balance, mu(z) u' = -g (z - H/2), so the steady profile is
    # the single-viscosity parabola, with the wall slip of the outer tau, in
    # the outer layers, and a parabola of curvature -g/nu_in inside.  (The
    # jump of relaxation time shifts the inner parabola by a constant, which
    # is not pinned here.)
    H, n, g = 24, 4, 1e-5
    tau_out, tau_in, k1, k2 = 0.8, 1.4, 8, 16
    mask = np.zeros((H, n, n), np.uint8)
    mask[k1:k2] = 1
    f = np.broadcast_to(W[:, None, None, None], (19, H, n, n)).copy()
    for _ in range(30000):
        f, rho, u = oracle.lb_step(f, tau_out, 0, None, (g, 0, 0), inside=mask, tau_in=tau_in)
    ux = u[0, :, 0, 0]
    nu_o, nu_i = (tau_out - 0.5) / 3, (tau_in - 0.5) / 3
    z = np.arange(H) + 0.5
    slip = g * (16 * (tau_out - 0.5) ** 2 - 3) / (24 * nu_o)
    outer = g / nu_o * (H * z / 2 - z * z / 2) + slip
    sel = (z < k1) | (z > k2)
    assert np.abs(ux[sel] - outer[sel]).max() < 1e-9 * outer.max()
    d2 = ux[k1:k2 - 2] - 2 * ux[k1 + 1:k2 - 1] + ux[k1 + 2:k2]
    assert np.allclose(d2, -g / nu_i, rtol=1e-7, atol=0)
    assert np.allclose(ux, ux[::-1], rtol=1e-12, atol=0)
