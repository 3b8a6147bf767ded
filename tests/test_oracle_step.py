"""Whole-step pins of the oracle: conservation laws and the Laplace pressure
jump of a free droplet (paper Sec. 2 and Fig. 1, pressure in units of the
Laplace pressure).  CPU only."""
import math

import numpy as np

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
