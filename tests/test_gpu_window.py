"""Whole-step parity at the 512x512x256 sixteen-droplet size (67 M cells),
through the C ABI, on windows of the box.

After 20 GPU steps (graph replay, autotuned launch, as the bench runs the
box) the GPU's own state (populations of each window plus a
one-cell halo, and every droplet's nodes) is advanced one step by the FP64
oracle: forces of every droplet (Eqs. 9-11), spreading into the whole box
(Eq. 8), the stream-collide with the Guo source on the window box (Eqs. 1-6;
the halo ring, which the oracle's periodic window box gets wrong, is dropped)
and the interpolation of the oracle's velocity at the nodes (Eq. 7) with the
forward Euler advection.  The GPU's next step must agree element by element
in the window interior, to FP32 rounding: populations (relative L2 of the
deviations) within 1e-5, band velocities within 1e-5 of their largest, node
positions within 1e-6 lu.  Each window spans the full height (both walls),
holds one droplet whole with its stencils, and crosses a periodic side of
the box; the other droplets' stencils stay out of it.

The same in FP16 deviation storage (scale 4096, as the bench runs it): the
oracle starts from the GPU's stored state, which it reads exactly, so the
velocities and nodes keep the FP32 bounds; each stored deviation of the new
state is the FP32 result rounded to FP16, within 2^-11 of it relatively
(half an ulp of an 11-bit significand; the scaled deviations lie in FP16's
normal range), so the populations are held to 2^-11 + 1e-5 = 5e-4.
"""
import numpy as np
import pytest

import oracle
from iblb_inputs import configs

from _helpers import deviation, lib_to_oracle_perm, rel_l2, say, to_oracle

pytestmark = pytest.mark.gpu

F32, F16, GRAPH, AUTOTUNE = 1, 2, 1, 2
STEPS = 20
# (droplet on the 4x4 grid, window lo x/y, window extent x/y)
WINDOWS = (
    ((3, 0), (400, 20), (120, 88)),   # crosses x = 512 -> 0
    ((1, 3), (150, 404), (84, 116)),  # crosses y = 512 -> 0
)


def _take(a, lo, ext, n, axis):
    return np.take(a, (np.arange(ext) + lo) % n, axis=axis)


@pytest.mark.parametrize("storage,scale,tol_f", [(F32, 1.0, 1e-5), (F16, 4096.0, 5e-4)])
def test_multidroplet_step_on_windows_matches_oracle(storage, scale, tol_f):
    import paper_2604_17463_amd as P
    say("512x512x256 sixteen droplets: one step on windows against the oracle, storage", storage)
    wl = configs.multidroplet_c5()
    box = wl.boxes[0]
    nx, ny, nz = box.nx, box.ny, box.nz
    perm = lib_to_oracle_perm()
    # graphs and the autotuned launch, as the bench runs this box
    s = P.Simulation(wl, storage=storage, flags=GRAPH | AUTOTUNE, dev_scale=scale)
    s.step(STEPS)
    q0 = [s.read_nodes(d) for d in range(len(wl.droplets))]
    halo = []
    for _, (x0, y0), (ex, ey) in WINDOWS:
        halo.append(to_oracle(s.read_window((x0 - 1, y0 - 1, 0), (ex + 2, ey + 2, nz)), perm))
    s.step(1)
    got = [s.read_window((x0, y0, 0), (ex, ey, nz), want_u=True) for _, (x0, y0), (ex, ey) in WINDOWS]
    q1 = [s.read_nodes(d) for d in range(len(wl.droplets))]
    drops, boxes = s.observables()
    assert boxes[0]["status_bits"] == 0
    s.close()

    # the oracle's step from the GPU's state: forces and spreading of every
    # droplet over the whole box
    F = np.zeros((3, nz, ny, nx))
    for d, dr in enumerate(wl.droplets):
        A = oracle.wetting_A(dr.sigma, dr.theta_eq, dr.xi, dr.n_exp, dr.m_exp)
        V0 = oracle.volume(dr.tris, dr.nodes)
        phi = oracle.node_forces(dr.tris, q0[d], dr.sigma, A, dr.xi, dr.n_exp, dr.m_exp, dr.k_vol, V0)
        assert phi["below_wall"] == 0
        oracle.spread((nz, ny, nx), box.zbc, q0[d], phi["phi"], F)
    for k, (((gi, gj), (x0, y0), (ex, ey)), hw, (fg, ug)) in enumerate(zip(WINDOWS, halo, got)):
        say(f"window {k}: x {x0}+{ex}, y {y0}+{ey}, all z")
        Fw = _take(_take(F, x0 - 1, ex + 2, nx, 3), y0 - 1, ey + 2, ny, 2)
        fn, _, u = oracle.lb_step(hw, box.tau, box.zbc, np.ascontiguousarray(Fw), box.body_force)
        f_ref = fn[:, :, 1:-1, 1:-1]
        u_ref = u[:, :, 1:-1, 1:-1]
        f_gpu = to_oracle(fg, perm)
        err_f = rel_l2(deviation(f_gpu), deviation(f_ref))
        say(f"window {k}: populations {err_f:.3e}")
        assert err_f < tol_f, (k, err_f)
        band = np.isfinite(ug[0])
        assert band.sum() > 1000, "the window holds the droplet's band"
        err_u = np.abs(ug[:, band] - u_ref[:, band]).max() / np.abs(u_ref[:, band]).max()
        say(f"window {k}: band velocities {err_u:.3e}")
        assert err_u < 1e-5, (k, err_u)
        # the droplet of this window: interpolation of the oracle's velocity
        # (window coordinates: the node stencils lie inside the interior)
        d = _droplet_at(wl, gi, gj)
        qw = q0[d] - np.array([x0 - 1, y0 - 1, 0.0])
        qw[:, 0] = np.mod(qw[:, 0], nx)
        qw[:, 1] = np.mod(qw[:, 1], ny)
        assert qw[:, 0].min() > 3 and qw[:, 0].max() < ex - 2
        assert qw[:, 1].min() > 3 and qw[:, 1].max() < ey - 2
        U = oracle.interp(np.ascontiguousarray(u), box.zbc, qw)
        err_q = np.abs(q1[d] - (q0[d] + U)).max()
        say(f"window {k}: nodes {err_q:.3e} lu")
        assert err_q < 1e-6, (k, err_q)


def _droplet_at(wl, gi, gj):
    """Index of the droplet centred at (64 + 128 gi, 64 + 128 gj)."""
    for d, dr in enumerate(wl.droplets):
        c = dr.nodes.mean(axis=0)
        if abs(c[0] - (64 + 128 * gi)) < 8 and abs(c[1] - (64 + 128 * gj)) < 8:
            return d
    raise AssertionError("no droplet at grid place %d, %d" % (gi, gj))
