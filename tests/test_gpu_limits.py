"""The largest boxes the library accepts: ten population planes within 4 GiB
(the 2-byte bulk path and the band kernel address them with 32-bit buffer
offsets).  A z-periodic box just below the limit, at rest, driven by a
uniform body force g, with a force-free droplet (sigma = 0, theta = 180 deg)
near the top, so that the band and interpolation kernels work at the
highest offsets.  Closed forms (Guo forcing adds g to every cell's momentum
each step): after n steps the bare momentum is n g everywhere, the mass is
unchanged, and the nodes, carried by u = (k + 1/2) g in step k, have moved
by n^2 g / 2."""
import numpy as np
import pytest

from iblb_inputs import mesh
from iblb_inputs.configs import Box, Droplet, Workload

from _helpers import say

pytestmark = pytest.mark.gpu

F32, F16 = 1, 2
LIMIT = 0xFFFFFFFF  # bytes of ten planes


# tolerances: FP32 storage rounds deviations to 2^-24, FP16 (times 4096) to
# 2^-11 of their size; the mass carries that rounding summed over 2e8 cells
@pytest.mark.parametrize("storage,elem,tol,mtol", [(F32, 4, 1e-5, 1e-9), (F16, 2, 2e-3, 1e-7)])
def test_box_at_the_plane_group_limit(storage, elem, tol, mtol):
    import paper_2604_17463_amd as P
    nx = ny = 448
    nz = LIMIT // (10 * elem * nx * ny)
    assert 10 * elem * nx * ny * nz <= LIMIT < 10 * elem * nx * ny * (nz + 1)
    g = 1e-5
    v, t = mesh.sphere(2, 4.0, (nx / 2.0, ny / 2.0, nz - 8.0))
    d = Droplet(0, v, t, sigma=0.0, theta_eq=np.pi, xi=0.2, k_vol=0.0)
    wl = Workload("limit", [Box(nx, ny, nz, tau=0.9, zbc=1, body_force=(g, 0.0, 0.0))], [d],
                  storage=storage)
    say("plane-group limit", storage, nx, ny, nz)
    s = P.Simulation(wl, storage=storage, flags=1, dev_scale=4096.0 if storage == F16 else 1.0)
    q0 = s.read_nodes(0)
    n = 4
    s.step(n)
    drops, boxes = s.observables()
    cells = nx * ny * nz
    assert boxes[0]["status_bits"] == 0
    assert abs(boxes[0]["mass"] / cells - 1.0) < mtol
    assert abs(boxes[0]["max_u"] / (n * g) - 1.0) < tol
    shift = s.read_nodes(0) - q0
    assert np.abs(shift[:, 0] / (n * n * g / 2) - 1.0).max() < tol
    assert np.abs(shift[:, 1:]).max() < tol * n * n * g
    s.close()
