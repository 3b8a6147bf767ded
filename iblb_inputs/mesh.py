"""Synthetic droplet meshes: icospheres, spheres placed over the wall, caps.

These are inputs only.  Nothing here evaluates a force, a volume, an area or
any other quantity of the method; both the oracle and the GPU library take the
arrays produced here and compute everything themselves.

Meshes are closed, consistently oriented triangulations whose triangles are
counter-clockwise seen from outside (the normal of (b-a)x(c-a) points out of
the droplet), which is the orientation the interface model of the paper's
Sec. 2 assumes for the outward normal n.
"""
from __future__ import annotations

import functools

import numpy as np

# The 12 vertices and 20 faces of a regular icosahedron (golden-ratio
# construction).  The faces are re-oriented below, so their listed order
# does not matter.
_PHI = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array(
    [
        (-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
        (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
        (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1),
    ],
    dtype=np.float64,
)
_ICO_F = np.array(
    [
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
    ],
    dtype=np.int64,
)


def _orient_outward(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Swap two corners of every face whose winding points toward the centre
    (unit-sphere meshes centred at the origin only)."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    f = f.copy()
    flip = s < 0
    f[flip, 1], f[flip, 2] = f[flip, 2].copy(), f[flip, 1].copy()
    return f


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere after `level` 4:1 subdivisions (fresh copies).

    Returns (nodes (N,3) float64, tris (T,3) int32) with N = 10*4^L + 2 and
    T = 20*4^L.  New vertices are edge midpoints pushed onto the unit sphere;
    numbering is deterministic (original vertices first, then midpoints in the
    order edges are met while walking the faces)."""
    v, f = _icosphere_cached(int(level))
    return v.copy(), f.copy()


@functools.lru_cache(maxsize=None)
def _icosphere_cached(level: int) -> tuple[np.ndarray, np.ndarray]:
    if level < 0:
        raise ValueError("level must be >= 0")
    v = [tuple(p / np.linalg.norm(p)) for p in _ICO_V]
    f = _orient_outward(np.array(v), _ICO_F)
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.add(v[i], v[j])
                p = p / np.linalg.norm(p)
                v.append(tuple(p))
                k = len(v) - 1
                cache[key] = k
            return k

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    return np.array(v, dtype=np.float64), f.astype(np.int32)


def geodesic(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit geodesic sphere of frequency `freq`: every icosahedron face is cut
    into freq^2 triangles on a regular barycentric grid and the grid points
    are pushed onto the unit sphere.  N = 10 freq^2 + 2 nodes, T = 20 freq^2
    triangles (freq = 2^L gives the level-L icosphere's counts; freq = 77
    gives 118,580 triangles).  Points on shared edges and corners are merged
    by their integer barycentric weights on the 12 icosahedron vertices."""
    n = int(freq)
    if n < 1:
        raise ValueError("freq must be >= 1")
    base = np.array([p / np.linalg.norm(p) for p in _ICO_V])
    faces = _orient_outward(base, _ICO_F)
    index: dict[tuple, int] = {}
    pts: list[np.ndarray] = []

    def node(a: int, b: int, c: int, i: int, j: int) -> int:
        w = {}
        for vid, wt in ((a, n - i - j), (b, i), (c, j)):
            if wt:
                w[vid] = w.get(vid, 0) + wt
        key = tuple(sorted(w.items()))
        k = index.get(key)
        if k is None:
            p = sum(base[vid] * wt for vid, wt in key) / n
            pts.append(p / np.linalg.norm(p))
            k = len(pts) - 1
            index[key] = k
        return k

    tris = []
    for a, b, c in faces:
        g = {(i, j): node(a, b, c, i, j) for i in range(n + 1) for j in range(n + 1 - i)}
        for i in range(n):
            for j in range(n - i):
                tris.append((g[(i, j)], g[(i + 1, j)], g[(i, j + 1)]))
                if i + j + 2 <= n:
                    tris.append((g[(i + 1, j)], g[(i + 1, j + 1)], g[(i, j + 1)]))
    v = np.array(pts, dtype=np.float64)
    f = _orient_outward(v, np.array(tris, dtype=np.int64))
    return v, f.astype(np.int32)


def sphere(level: int, radius: float, centre) -> tuple[np.ndarray, np.ndarray]:
    """Icosphere scaled to `radius` and moved to `centre`."""
    v, f = icosphere(level)
    return v * float(radius) + np.asarray(centre, dtype=np.float64), f


def _place_above_wall(v, radius: float, x: float, y: float, gap: float):
    v = v * float(radius)
    v[:, 0] += x
    v[:, 1] += y
    v[:, 2] += gap - v[:, 2].min()
    return v


def sphere_above_wall(level: int, radius: float, x: float, y: float, gap: float):
    """Sphere whose lowest node sits at height `gap` above the wall z = 0."""
    v, f = icosphere(level)
    return _place_above_wall(v, radius, x, y, gap), f


def geodesic_above_wall(freq: int, radius: float, x: float, y: float, gap: float):
    """The same with the geodesic sphere of frequency `freq`."""
    v, f = geodesic(freq)
    return _place_above_wall(v, radius, x, y, gap), f


def cap_radius(radius: float, theta0: float) -> float:
    """Radius of the spherical cap with contact angle theta0 (rad) that holds
    the same volume as a sphere of `radius` (plain solid geometry)."""
    c = np.cos(theta0)
    return float(radius * (4.0 / (2.0 - 3.0 * c + c ** 3)) ** (1.0 / 3.0))


def cap_on_wall(level: int, radius: float, theta0: float, x: float, y: float,
                base: float):
    """Spherical cap of contact angle theta0 standing on the plane z = base.

    A sphere of the cap radius is centred at height base - Rc*cos(theta0) and
    every node below the plane is lifted vertically onto it (only its z
    changes), which flattens the part under the plane into a disc while the
    triangulation keeps its orientation."""
    rc = cap_radius(radius, theta0)
    v, f = icosphere(level)
    v = v * rc
    v[:, 0] += x
    v[:, 1] += y
    v[:, 2] += base - rc * np.cos(theta0)
    below = v[:, 2] < base
    v[below, 2] = base
    return v, f


def cap_geodesic(freq: int, radius: float, theta0: float, x: float, y: float, base: float):
    """Spherical cap of contact angle theta0 on the plane z = base, holding
    the volume of a sphere of `radius`, meshed from the geodesic sphere of
    frequency `freq` with node density about even over the cap and its base
    disc.  A unit-sphere node at polar angle phi (from +z) and azimuth psi goes
    onto the cap at polar angle theta0 * phi / phi_s when phi <= phi_s, else
    onto the disc at radius a (pi - phi) / (pi - phi_s) (a = Rc sin theta0);
    phi_s splits the sphere's area in the ratio of cap area to disc area."""
    rc = cap_radius(radius, theta0)
    v, f = geodesic(freq)
    cap_area = 2.0 * np.pi * rc * rc * (1.0 - np.cos(theta0))
    a = rc * np.sin(theta0)
    disc_area = np.pi * a * a
    # (1 - cos phi_s) / 2 = cap_area / (cap_area + disc_area)
    phi_s = np.arccos(1.0 - 2.0 * cap_area / (cap_area + disc_area))
    phi = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    psi = np.arctan2(v[:, 1], v[:, 0])
    out = np.empty_like(v)
    on_cap = phi <= phi_s
    al = theta0 * phi[on_cap] / phi_s
    zc = base - rc * np.cos(theta0)       # centre of the cap's sphere
    out[on_cap, 0] = rc * np.sin(al) * np.cos(psi[on_cap])
    out[on_cap, 1] = rc * np.sin(al) * np.sin(psi[on_cap])
    out[on_cap, 2] = zc + rc * np.cos(al)
    rd = a * (np.pi - phi[~on_cap]) / (np.pi - phi_s)
    out[~on_cap, 0] = rd * np.cos(psi[~on_cap])
    out[~on_cap, 1] = rd * np.sin(psi[~on_cap])
    out[~on_cap, 2] = base
    out[:, 0] += x
    out[:, 1] += y
    return out, f


def is_closed_oriented(tris: np.ndarray) -> bool:
    """True when every directed edge occurs once and its reverse occurs once
    (closed, manifold, consistently oriented)."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    fwd = set(map(tuple, e))
    if len(fwd) != len(e):
        return False
    return all((b, a) in fwd for a, b in fwd)
