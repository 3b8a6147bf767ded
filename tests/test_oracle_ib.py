"""Pins of the oracle's immersed-boundary coupling (paper Sec. 2, Eqs. 7-8):
the discrete delta, spreading and interpolation, and the integer binning.
CPU only."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(99)


@pytest.mark.parametrize("r", list(RNG.uniform(0, 1, 8)) + [0.0, 0.5, 0.25])
def test_peskin_moment_conditions(r):
    # Peskin's 4-point function is built from: sum_k phi(r-k) = 1,
    # sum_k (r-k) phi(r-k) = 0 and sum_k phi(r-k)^2 = 3/8 for every shift r.
    ks = np.arange(-3, 4)
    w = np.array([oracle.peskin(r - k) for k in ks])
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(np.sum((r - ks) * w)) < 1e-15
    assert abs(np.sum(w * w) - 3.0 / 8.0) < 1e-15


def test_peskin_shape():
    assert oracle.peskin(0.0) == 0.5
    assert abs(oracle.peskin(1.0) - 0.25) < 1e-16
    assert oracle.peskin(2.0) == 0.0 and oracle.peskin(2.5) == 0.0
    assert oracle.peskin(-0.3) == oracle.peskin(0.3)
    # continuity at |r| = 1 and 2 from both branches
    e = 1e-9
    assert abs(oracle.peskin(1 - e) - oracle.peskin(1 + e)) < 1e-8
    assert abs(oracle.peskin(2 - e)) < 1e-4


def _nodes(n, lo, hi):
    return RNG.uniform(lo, hi, size=(n, 3))


def test_spread_conserves_force_and_first_moment():
    shape = (24, 20, 16)
    q = np.column_stack([RNG.uniform(4, 12, 50), RNG.uniform(4, 16, 50), RNG.uniform(4, 20, 50)])
    phi = RNG.standard_normal((50, 3))
    F, tw = oracle.spread(shape, 1, q, phi)
    assert np.allclose(F.sum(axis=(1, 2, 3)), phi.sum(0), rtol=0, atol=1e-13)
    assert np.all(tw == 0)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 for n in shape], indexing="ij")
    pos = np.stack([x, y, z])
    # sum_x x_a F_b = sum_j q_ja phi_jb (the kernel's first moment vanishes)
    lhs = np.einsum("aijk,bijk->ab", pos, F)
    rhs = q.T @ phi
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-11)


def test_spread_wraps_periodically_and_walls_absorb():
    shape = (8, 8, 8)
    q = np.array([[0.2, 7.9, 0.7], [5.0, 0.1, 7.6]])
    phi = np.array([[1.0, 2.0, 3.0], [-1.0, 0.5, 0.25]])
    F, tw = oracle.spread(shape, 0, q, phi)
    assert np.allclose(F.sum(axis=(1, 2, 3)) + tw, phi.sum(0), rtol=0, atol=1e-14)
    assert np.abs(tw).max() > 0.1  # some weight fell on the ghost layers
    Fp, twp = oracle.spread(shape, 1, q, phi)
    assert np.allclose(Fp.sum(axis=(1, 2, 3)), phi.sum(0), atol=1e-14) and np.all(twp == 0)


def test_interp_exact_for_linear_fields():
    shape = (20, 20, 20)
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 for n in shape], indexing="ij")
    a = np.array([0.1, -0.2, 0.3])
    B = RNG.standard_normal((3, 3)) * 0.01
    u = np.stack([a[c] + B[c, 0] * x + B[c, 1] * y + B[c, 2] * z for c in range(3)])
    q = _nodes(40, 4.0, 16.0)
    U = oracle.interp(u, 1, q)
    assert np.allclose(U, a + q @ B.T, rtol=0, atol=1e-14)


def test_interp_and_spread_are_adjoint():
    # sum_j U_j . phi_j = sum_x u(x) . F(x) with the same delta (Eqs. 7-8).
    shape = (12, 10, 9)
    for zbc in (0, 1):
        u = RNG.standard_normal((3,) + shape)
        q = np.column_stack([RNG.uniform(-3, 12, 30), RNG.uniform(-2, 13, 30),
                             RNG.uniform(0.3, 11.7, 30)])
        phi = RNG.standard_normal((30, 3))
        U = oracle.interp(u, zbc, q)
        F, _ = oracle.spread(shape, zbc, q, phi)
        assert abs(np.sum(U * phi) - np.sum(u * F)) < 1e-12


def test_interp_uses_zero_velocity_in_the_wall():
    shape = (8, 8, 8)
    u = np.ones((3,) + shape)
    q = np.array([[4.0, 4.0, 0.6], [4.0, 4.0, 4.0]])
    U = oracle.interp(u, 0, q)
    # at z = 0.6 cells k = -2, -1 are solid: weight lost = phi(2.1)+phi(1.1)
    lost = oracle.peskin(0.6 - (-1 + 0.5)) + oracle.peskin(0.6 - (-2 + 0.5))
    assert np.allclose(U[0], 1.0 - lost, atol=1e-15)
    assert np.allclose(U[1], 1.0, atol=1e-15)


def test_base_cells_brute_force():
    q = np.concatenate([RNG.uniform(-40, 60, (200, 3)),
                        np.array([[0.5, 1.5, 2.5], [-0.5, -1.0, 3.0], [31.5, 32.0, 0.49999999999]])])
    nx, ny = 32, 24
    b = oracle.base_cells(q, nx, ny)
    for j, p in enumerate(q):
        for a in range(3):
            # the unique integer with b + 1/2 <= q < b + 3/2
            cand = [k for k in range(-100, 100) if k + 0.5 <= p[a] < k + 1.5]
            assert len(cand) == 1
            want = cand[0]
            if a == 0:
                want %= nx
            if a == 1:
                want %= ny
            assert b[j, a] == want


@pytest.mark.parametrize("tile", [(4, 4, 4), (16, 4, 1), (3, 5, 2)])
def test_touched_tiles_brute_force(tile):
    shape = (16, 16, 12)
    nz, ny, nx = shape
    tx, ty, tz = tile
    q = np.column_stack([RNG.uniform(-5, 20, 25), RNG.uniform(0, 16, 25), RNG.uniform(0.2, 15.8, 25)])
    for zbc in (0, 1):
        flags = oracle.touched_tiles(q, shape, zbc, tile=tile)
        assert flags.shape == (-(-nz // tz), -(-ny // ty), -(-nx // tx))
        want = np.zeros_like(flags)
        for p in q:
            base = [int(np.floor(p[a] - 0.5)) for a in range(3)]
            for dz in range(-1, 3):
                k = base[2] + dz
                if zbc == 0 and not (0 <= k < nz):
                    continue
                for dy in range(-1, 3):
                    for dx in range(-1, 3):
                        want[(k % nz) // tz, ((base[1] + dy) % ny) // ty, ((base[0] + dx) % nx) // tx] = 1
        assert np.array_equal(flags, want)
