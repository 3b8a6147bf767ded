"""Time stepping of the FP64 oracle (test infrastructure only).

One step t -> t+1, in the order the paper's coupling implies (Sec. 2):
  1. nodal forces phi_j at the current node positions q^t     (Eqs. 9-11)
  2. spreading of phi onto the lattice, F^t                    (Eq. 8)
  3. moments with the half-force correction, BGK collision with
     the Guo source (relaxation time tau_in inside the droplets,
     tau outside, when the box sets tau_in), streaming with
     halfway bounce-back on resting or moving walls              (Eqs. 1-6)
  4. interpolation of u^t (the velocity of step 3) at q^t      (Eq. 7)
  5. forward Euler advection q^{t+1} = q^t + U                 (Sec. 2)
"""
from __future__ import annotations

import numpy as np

from . import (deformation, inside, interp, lattice, lb_step, mass, max_u, mesh_observables,
               node_forces, spread, volume, wetting_A)


class OracleSim:
    def __init__(self, workload, f0=None):
        self.wl = workload
        self.boxes = list(workload.boxes)
        self.drops = list(workload.droplets)
        self.c, self.w, self.opp = lattice()
        self.f = []
        for bi, b in enumerate(self.boxes):
            if f0 is not None and f0[bi] is not None:
                f = np.array(f0[bi], dtype=np.float64)
            else:
                f = np.empty((19, b.nz, b.ny, b.nx))
                f[:] = (self.w * b.rho0)[:, None, None, None]
            self.f.append(f)
        self.q = [np.array(d.nodes, dtype=np.float64) for d in self.drops]
        self.A = [wetting_A(d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp) for d in self.drops]
        self.V0 = [volume(d.tris, d.nodes) for d in self.drops]
        self.step_count = 0
        self._scratch = [np.empty_like(f) for f in self.f]
        self._spare = [np.empty_like(f) for f in self.f]
        self.last_phi = [None] * len(self.drops)
        self.last_F = [None] * len(self.boxes)
        self.last_u = [None] * len(self.boxes)
        self.last_rho = [None] * len(self.boxes)
        self.below_wall = 0

    def forces(self, di):
        d = self.drops[di]
        out = node_forces(d.tris, self.q[di], d.sigma, self.A[di], d.xi, d.n_exp,
                          d.m_exp, d.k_vol, self.V0[di])
        self.below_wall += out["below_wall"]
        return out["phi"]

    def inside_mask(self, bi):
        """Cells of box bi inside one of its droplets (at the current q)."""
        b = self.boxes[bi]
        ds = [i for i, d in enumerate(self.drops) if d.box == bi]
        tris, qs, off = [], [], 0
        for di in ds:
            tris.append(np.asarray(self.drops[di].tris, dtype=np.int32) + off)
            qs.append(self.q[di])
            off += len(self.q[di])
        return inside((b.nz, b.ny, b.nx), np.concatenate(tris), np.concatenate(qs))

    def step(self, n: int = 1):
        for _ in range(n):
            for bi, b in enumerate(self.boxes):
                ds = [i for i, d in enumerate(self.drops) if d.box == bi]
                F = np.zeros((3, b.nz, b.ny, b.nx))
                phis = {}
                for di in ds:
                    phis[di] = self.forces(di)
                for di in ds:
                    spread((b.nz, b.ny, b.nx), b.zbc, self.q[di], phis[di], F)
                mask = None
                tau_in = getattr(b, "tau_in", 0.0)
                if tau_in > 0.0 and ds:
                    mask = self.inside_mask(bi)
                uw = (tuple(getattr(b, "wall_lo", (0.0, 0.0))), tuple(getattr(b, "wall_hi", (0.0, 0.0))))
                moving = any(v != 0.0 for w in uw for v in w)
                fn, rho, u = lb_step(self.f[bi], b.tau, b.zbc, F, b.body_force,
                                     scratch=self._scratch[bi], out=self._spare[bi],
                                     inside=mask, tau_in=tau_in,
                                     u_wall=uw if moving else None, rho_wall=b.rho0)
                self._spare[bi] = self.f[bi]
                for di in ds:
                    U = interp(u, b.zbc, self.q[di])
                    self.q[di] = self.q[di] + U
                    self.last_phi[di] = phis[di]
                self.f[bi] = fn
                self.last_F[bi], self.last_u[bi], self.last_rho[bi] = F, u, rho
            self.step_count += 1

    def observables(self):
        per_drop = []
        for di, d in enumerate(self.drops):
            o = mesh_observables(d.tris, self.q[di], d.xi)
            dfm = deformation(d.tris, self.q[di])
            o["deformation"], o["inclination"] = dfm["D"], dfm["inclination"]
            o["step"] = self.step_count
            per_drop.append(o)
        per_box = [{"step": self.step_count, "mass": mass(f), "max_u": max_u(f)}
                   for f in self.f]
        return per_drop, per_box
