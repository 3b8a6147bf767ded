"""Whole-step pins of the oracle: conservation laws, the Laplace pressure
jump of a free droplet (paper Sec. 2 and Fig. 1, pressure in units of the
Laplace pressure) and the equilibrium spherical cap of a sessile droplet
(Eq. 11 and the steady heights of Sec. 3).  CPU only."""
import math

import numpy as np
import pytest

import oracle
from iblb_inputs import configs

C, W, _ = oracle.lattice()


def test_plain_c1_conserves_mass_and_stays_above_wall():
    wl = configs.plain_c1()
    sim = oracle.OracleSim(wl)
    m0 = oracle.mass(sim.f[0])
    z0 = sim.q[0][:, 2].min()
    sim.step(20)
    drops, boxes = sim.observables()
    assert abs(boxes[0]["mass"] - m0) < 1e-12 * m0
    assert sim.below_wall == 0
    # the wetting potential at d > xi pulls the lowest nodes toward the wall
    assert drops[0]["z_min"] < z0
    assert drops[0]["z_min"] > wl.droplets[0].xi


def _laplace_run(steps):
    wl = configs.free_droplet(n=32, r=8.0, level=3, tau=1.0, sigma=0.01)
    sim = oracle.OracleSim(wl)
    sim.step(steps)
    return wl, sim


def test_free_droplet_laplace_jump_and_zero_momentum():
    # Steady free droplet: c_s^2 (<rho>_in - <rho>_out) = 2 sigma / R_eq with
    # R_eq the radius of the sphere of the mesh's volume; averages are taken
    # 3 lu away from the diffuse interface.  The IB interface is smeared over
    # the 4-cell stencil, hence a few percent of tolerance.  Surface tension
    # is an internal force, so the total fluid momentum stays zero.
    wl, sim = _laplace_run(750)
    f = sim.f[0]
    rho = f.sum(0)
    nz, ny, nx = rho.shape
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 for n in (nz, ny, nx)], indexing="ij")
    q = sim.q[0]
    cen = q.mean(0)
    r = np.sqrt((x - cen[0]) ** 2 + (y - cen[1]) ** 2 + (z - cen[2]) ** 2)
    V = oracle.volume(wl.droplets[0].tris, q)
    req = (3 * V / (4 * math.pi)) ** (1 / 3)
    dp = (rho[r < req - 3].mean() - rho[r > req + 3].mean()) / 3.0
    assert abs(dp / (2 * 0.01 / req) - 1.0) < 0.03
    mom = np.einsum("qa,qijk->a", C, f)
    assert np.abs(mom).max() < 1e-10
    # the centre does not drift
    assert np.abs(cen - 16.0).max() < 1e-9


@pytest.mark.slow
def test_sessile_droplet_relaxes_to_the_spherical_cap_of_theta_eq():
    # A sphere resting at height xi above the wall, with the wetting amplitude
    # A of Eq. 11 for theta_eq = 90 degrees, relaxes to the spherical cap of
    # its volume: h / R0 = (1 - cos t) (4 / (2 - 3 cos t + cos^3 t))^(1/3)
    # (1.2599 at 90 degrees, R0 the equal-volume sphere radius) and apparent
    # angle 2 atan(h / r_c) = theta_eq.  The film below the droplet keeps the
    # shape slightly above the ideal cap (the paper's own run sits 3.4 % above
    # it at xi / R0 = 0.05); 5 % on h / R0 and 5 degrees on the angle.  xi
    # here is one lattice unit (xi / R0 = 0.1): at xi below one cell the
    # interaction is not resolved by the 4-cell delta function and the
    # apparent angle stays far above theta_eq.
    from iblb_inputs import mesh
    from iblb_inputs.configs import Box, Droplet, Workload
    R, xi, theta = 10.0, 1.0, math.radians(90.0)
    v, t = mesh.sphere_above_wall(4, R, 20.0, 20.0, xi)
    wl = Workload("cap-equilibrium", [Box(40, 40, 28, tau=1.0)],
                  [Droplet(0, v, t, sigma=0.01, theta_eq=theta, xi=xi, k_vol=2 * 0.01 / R)])
    sim = oracle.OracleSim(wl)
    sim.step(8000)
    d = sim.observables()[0][0]
    R0 = (3 * d["volume"] / (4 * math.pi)) ** (1 / 3)
    c = math.cos(theta)
    ideal = (1 - c) * (4 / (2 - 3 * c + c ** 3)) ** (1 / 3)
    assert abs(d["height"] / R0 / ideal - 1.0) < 0.05, d["height"] / R0
    theta_app = 2 * math.atan(d["height"] / d["contact_radius"])
    assert abs(math.degrees(theta_app - theta)) < 5.0, math.degrees(theta_app)
