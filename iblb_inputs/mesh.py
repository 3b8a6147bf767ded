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


def sphere(level: int, radius: float, centre) -> tuple[np.ndarray, np.ndarray]:
    """Icosphere scaled to `radius` and moved to `centre`."""
    v, f = icosphere(level)
    return v * float(radius) + np.asarray(centre, dtype=np.float64), f


def sphere_above_wall(level: int, radius: float, x: float, y: float, gap: float):
    """Sphere whose lowest node sits at height `gap` above the wall z = 0."""
    v, f = icosphere(level)
    v = v * float(radius)
    v[:, 0] += x
    v[:, 1] += y
    v[:, 2] += gap - v[:, 2].min()
    return v, f


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


def is_closed_oriented(tris: np.ndarray) -> bool:
    """True when every directed edge occurs once and its reverse occurs once
    (closed, manifold, consistently oriented)."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    fwd = set(map(tuple, e))
    if len(fwd) != len(e):
        return False
    return all((b, a) in fwd for a, b in fwd)
