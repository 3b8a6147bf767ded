"""Pins of the oracle's lattice Boltzmann part (paper Sec. 2, Eqs. 1-6)
against closed forms and exact invariants.  CPU only."""
import math

import numpy as np
import pytest

import oracle

C, W, OPP = oracle.lattice()
RNG = np.random.default_rng(1234)


def test_velocity_set_isotropy():
    # D3Q19 textbook moments: sum w = 1, sum w c = 0, sum w c c = cs^2 I,
    # sum w c c c c = cs^4 (d d + d d + d d), cs^2 = 1/3.
    assert len(set(map(tuple, C))) == 19
    assert abs(W.sum() - 1.0) < 1e-15
    assert np.allclose(W @ C, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", W, C, C), np.eye(3) / 3, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(m4, iso, atol=1e-16)
    for i in range(19):
        assert np.array_equal(C[OPP[i]], -C[i])


@pytest.mark.parametrize("trial", range(5))
def test_equilibrium_moments(trial):
    rho = 1.0 + 0.1 * RNG.standard_normal()
    u = 0.05 * RNG.standard_normal(3)
    fe = oracle.feq(rho, u)
    assert abs(fe.sum() - rho) < 1e-15 * 10
    assert np.allclose(C.T @ fe, rho * u, rtol=0, atol=1e-15)
    pi = np.einsum("i,ia,ib->ab", fe, C, C)
    assert np.allclose(pi, rho * np.eye(3) / 3 + rho * np.outer(u, u), rtol=0, atol=1e-15)


def test_equilibrium_at_rest_is_weights():
    assert np.array_equal(oracle.feq(1.0, np.zeros(3)), W)


@pytest.mark.parametrize("trial", range(5))
def test_guo_source_moments(trial):
    tau = 0.55 + RNG.uniform(0, 1.5)
    u = 0.05 * RNG.standard_normal(3)
    F = 1e-3 * RNG.standard_normal(3)
    S = oracle.guo(tau, u, F)
    pre = 1.0 - 1.0 / (2.0 * tau)
    assert abs(S.sum()) < 1e-18
    assert np.allclose(C.T @ S, pre * F, rtol=0, atol=1e-18)
    second = np.einsum("i,ia,ib->ab", S, C, C)
    assert np.allclose(second, pre * (np.outer(u, F) + np.outer(F, u)), rtol=0, atol=1e-18)


def test_moments_half_force_correction():
    rho0, u0 = 1.02, np.array([0.01, -0.02, 0.005])
    F = np.array([1e-3, 2e-3, -3e-3])
    rho, u = oracle.moments(oracle.feq(rho0, u0), F)
    assert abs(rho - rho0) < 1e-15
    assert np.allclose(u, u0 + F / (2 * rho0), rtol=0, atol=1e-16)


def _eq_field(rho, u):
    """f = f_eq(rho(x), u(x)) for fields rho (nz,ny,nx), u (3,nz,ny,nx)."""
    nz, ny, nx = rho.shape
    f = np.empty((19, nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                f[:, k, j, i] = oracle.feq(rho[k, j, i], u[:, k, j, i])
    return f


def test_rest_state_is_a_fixed_point():
    # f = w rho0 with no force stays put (to the rounding of sum w = 1).
    f = np.empty((19, 6, 5, 4))
    f[:] = W[:, None, None, None]
    for zbc in (0, 1):
        fn, rho, u = oracle.lb_step(f, 0.77, zbc)
        assert np.abs(fn - f).max() < 1e-16
        assert np.abs(u).max() < 1e-16


@pytest.mark.parametrize("zbc", [0, 1])
def test_mass_conserved_with_forcing(zbc):
    shape = (8, 6, 5)
    rho = 1.0 + 0.01 * RNG.standard_normal(shape)
    u = 0.02 * RNG.standard_normal((3,) + shape)
    f = _eq_field(rho, u) + 1e-4 * RNG.standard_normal((19,) + shape)
    F = 1e-3 * RNG.standard_normal((3,) + shape)
    m0 = f.sum()
    for _ in range(5):
        f, _, _ = oracle.lb_step(f, 0.7, zbc, F, (1e-4, 0, 0))
    assert abs(f.sum() - m0) < 1e-12 * m0


def test_streaming_moves_mass_centre_by_momentum():
    # Exact discrete identity of stream-after-collide: the displacement of
    # sum_x x rho over one step equals the post-collision momentum.  With the
    # half-force velocity inside f_eq and the Guo source that momentum is
    # sum c f + F (F/(2 tau) from relaxation plus (1 - 1/(2 tau)) F from S).
    # Fixes the direction of streaming and the force bookkeeping.
    shape = (16, 16, 16)
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 for n in shape], indexing="ij")
    bump = 0.01 * np.exp(-((x - 8) ** 2 + (y - 8) ** 2 + (z - 8) ** 2) / 2.0)
    u = np.zeros((3,) + shape)
    u[0] = 0.03 * bump / 0.01
    u[1] = -0.02 * bump / 0.01
    f = _eq_field(1.0 + bump, u)
    tau = 0.9
    F = np.zeros((3,) + shape)
    F[2] = 1e-4 * bump / 0.01
    fn, _, _ = oracle.lb_step(f, tau, 1, F)
    pos = np.stack([x, y, z]) - 8.0  # centred, keeps the sums well conditioned
    before = np.einsum("aijk,ijk->a", pos, f.sum(0))
    after = np.einsum("aijk,ijk->a", pos, fn.sum(0))
    mom = np.einsum("qa,qijk->a", C, f) + F.sum(axis=(1, 2, 3))
    # atol: rounding floor of 4096 cells x 19 populations weighted by |x| <= 8
    assert np.allclose(after - before, mom, rtol=1e-9, atol=5e-11)


def _poiseuille(tau, H=24, g=1e-6):
    nu = (tau - 0.5) / 3.0
    f = np.empty((19, H, 1, 1))
    f[:] = W[:, None, None, None]
    s, o2 = np.empty_like(f), np.empty_like(f)
    r, u = np.empty((H, 1, 1)), np.empty((3, H, 1, 1))
    n = int(36 * H * H / (math.pi ** 2 * nu))
    for _ in range(n):
        fn, _, _ = oracle.lb_step(f, tau, 0, None, (g, 0.0, 0.0), scratch=s, out=o2,
                                  rho=r, u=u)
        o2, f = f, fn
    return u[0, :, 0, 0].copy(), u, f


@pytest.mark.parametrize("tau", [0.8, 0.5 + math.sqrt(3) / 4, 1.0, 1.5])
def test_poiseuille_closed_form(tau):
    # Channel 0 < z < H between resting walls placed halfway between the
    # first/last fluid layer and the ghost layer, body force g along x.
    # For BGK with halfway bounce-back the steady profile is the parabola
    # g z (H - z) / (2 nu) plus a uniform slip (g/nu)(2 Lambda/3 - 1/8),
    # Lambda = (tau - 1/2)^2; the slip vanishes at Lambda = 3/16 (Ginzburg's
    # "magic" relaxation time tau = 1/2 + sqrt(3)/4).  nu = (tau - 1/2)/3.
    H, g = 24, 1e-6
    ux, u, f = _poiseuille(tau, H, g)
    nu = (tau - 0.5) / 3.0
    lam = (tau - 0.5) ** 2
    z = np.arange(H) + 0.5
    exact = g * z * (H - z) / (2 * nu) + (g / nu) * (2 * lam / 3 - 1.0 / 8.0)
    assert np.linalg.norm(ux - exact) / np.linalg.norm(exact) < 1e-10
    assert np.abs(u[1:]).max() < 1e-9 * np.abs(ux).max()
    assert abs(f.sum() - H) < 1e-11 * H  # ~2e4 steps of FP64 rounding


def test_shear_wave_decay_gives_paper_viscosities():
    # The paper prints mu for three relaxation times (golden file).  Measure
    # the viscosity of the oracle's dynamics from the decay of a periodic
    # shear wave u_x = U sin(k z): amplitude ~ exp(-nu k^2 t).
    rows = []
    re_row = None
    with open(__file__.replace("test_oracle_lattice.py", "golden/paper_viscosity.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            p = line.split()
            if p[0] == "RE":
                re_row = [float(v) for v in p[1:]]
            else:
                rows.append([float(v) for v in p])
    assert len(rows) == 3 and re_row is not None
    L = 64
    k = 2 * math.pi / L
    z = np.arange(L) + 0.5
    for tau, mu_printed, tol in rows:
        u = np.zeros((3, L, 1, 1))
        u[0, :, 0, 0] = 1e-4 * np.sin(k * z)
        f = _eq_field(np.ones((L, 1, 1)), u)

        def amp(fld):
            _, _, uu = oracle.lb_step(fld, tau, 1)
            return 2.0 / L * np.sum(uu[0, :, 0, 0] * np.sin(k * z))

        for _ in range(200):
            f, _, _ = oracle.lb_step(f, tau, 1)
        a1 = amp(f)
        n = 400
        for _ in range(n):
            f, _, _ = oracle.lb_step(f, tau, 1)
        a2 = amp(f)
        nu = -math.log(a2 / a1) / (k * k * n)
        assert abs(nu - mu_printed) <= max(tol, 2e-3 * mu_printed), (tau, nu, mu_printed)
    sigma, R0, mu, re_printed, tol = re_row
    assert abs(sigma * R0 / mu ** 2 - re_printed) < tol


def _first_order_populations(rho, u):
    """f_i = w_i rho (1 + 3 c_i . u) per cell: by the lattice isotropy
    (sum w c = 0, sum w c c = I/3) its density is rho and its momentum rho u
    exactly, independently of the oracle's equilibrium."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    cu = np.einsum("ia,a...->i...", C.astype(np.float64), u)
    return W.reshape((19,) + (1,) * rho.ndim) * rho[None] * (1.0 + 3.0 * cu)


def test_max_u_of_a_uniform_field_is_its_velocity():
    # every cell carries the same (rho, U): max |sum c f| / rho = |U|
    shape = (3, 4, 5)
    U = np.array([0.03, -0.04, 0.012])
    rho = np.full(shape, 1.07)
    f = _first_order_populations(rho, np.broadcast_to(U[:, None, None, None], (3,) + shape))
    assert abs(oracle.max_u(f) - np.linalg.norm(U)) < 1e-15


def test_max_u_takes_the_largest_cell_and_divides_by_the_local_density():
    # two regions of different density and velocity; the largest speed sits
    # in the light region.  Dividing by a reference density instead of the
    # cell's own, or dropping a velocity component, picks the other region
    # or another value.
    shape = (4, 4, 6)
    rho = np.full(shape, 2.0)
    u = np.zeros((3,) + shape)
    u[0] = 0.05                                  # heavy region: |u| = 0.05, |j| = 0.1
    light = (slice(None), slice(None), slice(3, 5))
    rho[light] = 0.5
    u[:, light[0], light[1], light[2]] = np.array([0.02, -0.03, 0.06])[:, None, None, None]
    u[:, 1, 2, 4] = [0.0, 0.0, -0.071]           # one cell of the light region is the fastest
    f = _first_order_populations(rho, u)
    assert abs(oracle.max_u(f) - 0.071) < 1e-15
    # a fluid at rest has no velocity at any density
    assert oracle.max_u(_first_order_populations(rho, np.zeros_like(u))) == 0.0
