"""Seeded synthetic workloads shaped like the paper's spreading runs.

A workload is a list of lattice boxes and a list of droplets, each droplet
living in one box.  The five named workloads reproduce the box sizes, mesh
resolutions, contact angles, relaxation times and surface tensions of the
spreading experiments (paper Sec. 3 and Sec. 4: droplets of radius R0 with
xi/R0 = 0.05, mesh edges of about one lattice unit, a flat wetting wall at the
bottom, periodic sides) at sizes from a few thousand to 67 million cells.

Only input values are produced here: the wetting amplitude A, the volume V0,
the node normals and everything else the method computes are left to the
oracle and to the library.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from . import mesh as _mesh

Z_WALLS = 0
Z_PERIODIC = 1

F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
STORAGE_NAMES = {F64: "f64", F32: "f32", F16DEV: "f16dev", BF16DEV: "bf16dev"}


@dataclass
class Box:
    nx: int
    ny: int
    nz: int
    tau: float
    rho0: float = 1.0
    zbc: int = Z_WALLS
    body_force: tuple = (0.0, 0.0, 0.0)
    tau_in: float = 0.0        # relaxation time inside droplets (0: tau everywhere)
    wall_lo: tuple = (0.0, 0.0)  # (ux, uy) of the wall at z = 0
    wall_hi: tuple = (0.0, 0.0)  # (ux, uy) of the wall at z = nz

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Droplet:
    box: int
    nodes: np.ndarray          # (N,3) float64, unwrapped coordinates, wall at z = 0
    tris: np.ndarray           # (T,3) int32, counter-clockwise seen from outside
    sigma: float
    theta_eq: float            # rad
    xi: float
    n_exp: int = 9
    m_exp: int = 3
    k_vol: float = 0.0


@dataclass
class Workload:
    name: str
    boxes: list
    droplets: list
    steps: int = 1
    log_every: int = 0
    storage: int = F32
    dev_scale: float = 1.0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return sum(b.cells for b in self.boxes)

    @property
    def nodes(self) -> int:
        return sum(len(d.nodes) for d in self.droplets)

    def with_storage(self, storage: int, dev_scale: float | None = None) -> "Workload":
        if dev_scale is None:
            dev_scale = 4096.0 if storage == F16DEV else 1.0
        return replace(self, storage=storage, dev_scale=dev_scale)


def workload_hash(wl: Workload) -> str:
    """sha256 of everything that defines a workload's inputs (box sizes and
    parameters, meshes, droplet parameters): stored traces carry it, so that
    a trace is only compared with runs of the inputs it was made from."""
    import hashlib
    h = hashlib.sha256()
    for b in wl.boxes:
        h.update(repr((b.nx, b.ny, b.nz, b.tau, b.rho0, b.zbc, tuple(b.body_force))).encode())
    for d in wl.droplets:
        h.update(np.ascontiguousarray(d.nodes, dtype=np.float64).tobytes())
        h.update(np.ascontiguousarray(d.tris, dtype=np.int32).tobytes())
        h.update(repr((d.box, d.sigma, d.theta_eq, d.xi, d.n_exp, d.m_exp, d.k_vol)).encode())
    return h.hexdigest()


def _deg(a: float) -> float:
    return a * math.pi / 180.0


def plain_c1() -> Workload:
    """32x32x24 box, tau = 1, one level-3 icosphere (642 nodes) of radius 8
    centred 9 lu above the wetting wall, sigma = 0.01, theta_eq = 90 deg,
    xi = 0.05 R, no volume penalty, fluid at rest, 200 steps."""
    r = 8.0
    v, t = _mesh.sphere(3, r, (16.0, 16.0, 9.0))
    box = Box(32, 32, 24, tau=1.0)
    d = Droplet(0, v, t, sigma=0.01, theta_eq=_deg(90.0), xi=0.05 * r, k_vol=0.0)
    return Workload("plain-fp64-32x32x24-ico3", [box], [d], steps=200, storage=F64)


def spreading_c2(steps: int = 20000) -> Workload:
    """128x128x64 box, tau = 0.8, sigma = 0.005; a level-5 mesh (10242 nodes)
    holding the volume of a radius-24 sphere, started as a 150 deg cap and
    relaxing toward theta_eq = 60 deg; h and r_c logged every 100 steps."""
    r = 24.0
    xi = 0.05 * r
    v, t = _mesh.cap_on_wall(5, r, _deg(150.0), 64.0, 64.0, xi)
    box = Box(128, 128, 64, tau=0.8)
    sigma = 0.005
    d = Droplet(0, v, t, sigma=sigma, theta_eq=_deg(60.0), xi=xi, k_vol=2.0 * sigma / r)
    return Workload("spreading-fp32-128x128x64-ico5", [box], [d], steps=steps,
                    log_every=100, storage=F32)


def precision_c3(tau: float = 0.6, steps: int = 10000) -> Workload:
    """256x256x128 box, one level-6 sphere (40962 nodes) of radius 48 resting
    at height xi above the wall, theta_eq = 45 deg, sigma = 0.005."""
    r = 48.0
    xi = 0.05 * r
    v, t = _mesh.sphere_above_wall(6, r, 128.0, 128.0, xi)
    box = Box(256, 256, 128, tau=tau)
    sigma = 0.005
    d = Droplet(0, v, t, sigma=sigma, theta_eq=_deg(45.0), xi=xi, k_vol=2.0 * sigma / r)
    return Workload(f"precision-256x256x128-ico6-tau{tau:g}", [box], [d], steps=steps,
                    storage=F32)


def batched_c4(seed: int = 17463, n_boxes: int = 64, steps: int = 1000) -> Workload:
    """64 independent boxes of uneven sizes (48^3 up to 128x128x64), each with
    one sphere of radius U[10,24] (level 4 below 17, else level 5) resting at
    height xi, theta_eq U[30,150] deg, tau U[0.6,1.5], sigma = 0.005."""
    rng = np.random.default_rng(seed)
    sides = np.arange(48, 129, 16)
    heights = np.array([48, 56, 64])
    boxes, drops = [], []
    sigma = 0.005
    for b in range(n_boxes):
        lx = int(rng.choice(sides))
        ly = int(rng.choice(sides))
        lz = int(rng.choice(heights))
        while True:
            r = float(rng.uniform(10.0, 24.0))
            xi = 0.05 * r
            if 2 * r + 8 <= min(lx, ly) and 2 * r + xi + 6 <= lz:
                break
        level = 4 if r < 17.0 else 5
        theta = _deg(float(rng.uniform(30.0, 150.0)))
        tau = float(rng.uniform(0.6, 1.5))
        v, t = _mesh.sphere_above_wall(level, r, lx / 2.0, ly / 2.0, xi)
        boxes.append(Box(lx, ly, lz, tau=tau))
        drops.append(Droplet(b, v, t, sigma=sigma, theta_eq=theta, xi=xi,
                             k_vol=2.0 * sigma / r))
    return Workload(f"batched-{n_boxes}boxes-seed{seed}", boxes, drops, steps=steps,
                    storage=F32)


def multidroplet_c5(seed: int = 17464, steps: int = 5000) -> Workload:
    """512x512x256 box (67M cells), 16 level-5 spheres on a 4x4 grid of
    centres (64 + 128 i, 64 + 128 j), radii U[20,32], theta_eq U[40,120] deg,
    tau = 0.9, sigma = 0.005."""
    rng = np.random.default_rng(seed)
    box = Box(512, 512, 256, tau=0.9)
    drops = []
    sigma = 0.005
    for i in range(4):
        for j in range(4):
            r = float(rng.uniform(20.0, 32.0))
            xi = 0.05 * r
            theta = _deg(float(rng.uniform(40.0, 120.0)))
            v, t = _mesh.sphere_above_wall(5, r, 64.0 + 128.0 * i, 64.0 + 128.0 * j, xi)
            drops.append(Droplet(0, v, t, sigma=sigma, theta_eq=theta, xi=xi,
                                 k_vol=2.0 * sigma / r))
    return Workload("multidroplet-512x512x256-16xico5", [box], drops, steps=steps,
                    storage=F32)


def poiseuille(nx: int = 4, ny: int = 4, nz: int = 24, tau: float = 0.8,
               g: float = 1e-6) -> Workload:
    """Empty channel between the two walls driven by a body force along x."""
    return Workload(f"poiseuille-{nz}-tau{tau:g}", [Box(nx, ny, nz, tau=tau,
                    body_force=(g, 0.0, 0.0))], [], storage=F64)


def free_droplet(n: int = 32, r: float = 8.0, level: int = 3, tau: float = 1.0,
                 sigma: float = 0.01) -> Workload:
    """Droplet in a fully periodic box with no wall interaction (theta = 180
    deg makes the wetting amplitude vanish)."""
    v, t = _mesh.sphere(level, r, (n / 2.0, n / 2.0, n / 2.0))
    box = Box(n, n, n, tau=tau, zbc=Z_PERIODIC)
    d = Droplet(0, v, t, sigma=sigma, theta_eq=math.pi, xi=0.05 * r, k_vol=0.0)
    return Workload(f"free-droplet-{n}", [box], [d], storage=F64)


def paper_spreading(tau: float = 0.732, freq: int = 77, shape=(250, 250, 150), r0: float = 60.0,
                    sigma: float = 0.001, theta_eq_deg: float = 60.0, start: str = "cap",
                    storage: int = F32) -> Workload:
    """The spreading runs of the paper's Sec. 3 at their own scale: a droplet
    of volume 4/3 pi R0^3 (R0 = 60) standing as a 90 deg cap on the wall
    spreads toward theta_eq = 60 deg; 250 x 250 x 150 lattice, a geodesic
    mesh of 20 freq^2 triangles (freq = 77: 118,580, the paper's ~120,000),
    xi = 0.05 R0, sigma = 0.001, lambda = 1 with tau in {0.56, 0.59, 0.732,
    1.1}.  Time unit t_mu = mu R0 / sigma; the paper runs 50 t_mu and reports
    h / R0 -> 0.96 in the Stokes limit.  The volume penalty follows the other
    workloads (k_V = 2 sigma / R0).  start = "sphere" places the sphere of
    radius R0 with its lowest node at xi above the wall instead of the cap."""
    nx, ny, nz = shape
    xi = 0.05 * r0
    if start == "cap":
        v, t = _mesh.cap_geodesic(freq, r0, _deg(90.0), nx / 2.0, ny / 2.0, xi)
    elif start == "sphere":
        v, t = _mesh.geodesic_above_wall(freq, r0, nx / 2.0, ny / 2.0, xi)
    else:
        raise ValueError("start must be 'cap' or 'sphere'")
    box = Box(nx, ny, nz, tau=tau)
    d = Droplet(0, v, t, sigma=sigma, theta_eq=_deg(theta_eq_deg), xi=xi, k_vol=2.0 * sigma / r0)
    mu = (tau - 0.5) / 3.0
    name = f"paper-{'spreading' if start == 'cap' else 'sphere'}-{nx}x{ny}x{nz}-tau{tau:g}"
    if theta_eq_deg != 60.0:
        name += f"-theta{theta_eq_deg:g}"
    return Workload(name, [box], [d], storage=storage,
                    extra={"t_mu": mu * r0 / sigma, "r0": r0, "re": sigma * r0 / (mu * mu)})


def paper_cap45(storage: int = F32) -> Workload:
    """Sec. 4, first wetting case of the Basilisk comparison: the 90 deg cap of
    the Sec. 3 runs spreads toward theta_eq = 45 deg at tau = 0.59 (mu = 0.03,
    Re = 66.7) on the 250 x 250 x 150 lattice; the paper compares
    half-profiles at t / t_mu = 0, 4, 10, 70."""
    return paper_spreading(0.59, theta_eq_deg=45.0, storage=storage)


def paper_neck(storage: int = F32) -> Workload:
    """Sec. 4, inertial case: a sphere of radius R0 = 60 with its lowest node
    at xi above the wall spreads toward theta_eq = 45 deg at tau = 0.56
    (mu = 0.02, Re = 150) on a 300 x 300 x 250 lattice; a neck forms at the
    contact line, the droplet flattens and bounces back toward a cap (the
    paper shows profiles at t / t_mu = 3, 18, 30, 48)."""
    return paper_spreading(0.56, shape=(300, 300, 250), theta_eq_deg=45.0, start="sphere",
                           storage=storage)


def shear_droplet(lam: float = 1.0, r: float = 12.0, ca: float = 0.05, re: float = 0.01,
                  shape=(128, 96, 192), level: int = 5, tau_out: float = 1.0,
                  storage: int = F32) -> Workload:
    """Free droplet of radius r at the centre of a plane shear flow (paper
    Sec. 4): walls at z = 0 and z = nz move with -/+ gamma nz / 2 along x;
    viscosity ratio lam = (tau_in - 1/2) / (tau_out - 1/2); rho = 1.
    Re = gamma r^2 / nu_out and Ca = mu_out gamma r / sigma fix the shear
    rate gamma and sigma.  No wetting (theta = 180 deg) and no volume
    penalty.  The paper's own run: r = 19, Re = 0.01, Ca = 0.05, tau = 1."""
    nx, ny, nz = shape
    nu = (tau_out - 0.5) / 3.0
    gamma = re * nu / (r * r)
    sigma = nu * gamma * r / ca
    uw = gamma * nz / 2.0
    box = Box(nx, ny, nz, tau=tau_out, tau_in=0.5 + lam * (tau_out - 0.5),
              wall_lo=(-uw, 0.0), wall_hi=(uw, 0.0))
    v, t = _mesh.sphere(level, r, (nx / 2.0, ny / 2.0, nz / 2.0))
    d = Droplet(0, v, t, sigma=sigma, theta_eq=math.pi, xi=0.05 * r, k_vol=0.0)
    return Workload(f"shear-droplet-lam{lam:g}-{nx}x{ny}x{nz}-r{r:g}", [box], [d], storage=storage,
                    extra={"shear_rate": gamma, "ca": ca, "re": re, "lam": lam,
                           "t_cap": ca / gamma})


def perturbed_populations(box: Box, seed: int, amplitude: float = 1e-3) -> np.ndarray:
    """Random populations around the rest state, [19][nz][ny][nx] in the order
    of the velocity set passed later by the caller (weights w): returns a
    multiplicative noise field eta with f = w * rho0 * (1 + eta)."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal((19, box.nz, box.ny, box.nx))


def jitter_nodes(nodes: np.ndarray, seed: int, amplitude: float) -> np.ndarray:
    """Nodes moved by a seeded uniform offset in [-amplitude, amplitude]^3."""
    rng = np.random.default_rng(seed)
    return nodes + rng.uniform(-amplitude, amplitude, size=nodes.shape)


NAMED = {
    "c1": plain_c1,
    "c2": spreading_c2,
    "c3": precision_c3,
    "c4": batched_c4,
    "c5": multidroplet_c5,
}
