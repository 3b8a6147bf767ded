"""FP64 CPU oracle for the IBLB wetting step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It loads `liboracle.so`, built from `iblb_oracle.c` with gcc,
and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as _C
import os as _os
import subprocess as _sp

import numpy as _np

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_SRC = _os.path.join(_HERE, "iblb_oracle.c")
# IBLB_ORACLE_LIB names another build of iblb_oracle.c to load (the
# sanitizer test loads an ASan/UBSan build through it)
_LIB = _os.environ.get("IBLB_ORACLE_LIB") or _os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over z-slabs of the LB step)."""
    if force or not _os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        _sp.check_call(cmd)
        _os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _os.path.exists(_LIB):
            build()
        _lib = _C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = _np.ctypeslib.ndpointer(dtype=_np.float64, flags="C_CONTIGUOUS")
_ip = _np.ctypeslib.ndpointer(dtype=_np.int32, flags="C_CONTIGUOUS")
_bp = _np.ctypeslib.ndpointer(dtype=_np.uint8, flags="C_CONTIGUOUS")
_vp = _C.c_void_p
_i = _C.c_int
_d = _C.c_double


def _declare(L):
    L.orc_num_threads.restype = _i
    L.orc_set_threads.argtypes = [_i]
    L.orc_lattice.argtypes = [_ip, _dp, _ip]
    L.orc_feq.argtypes = [_d, _dp, _dp]
    L.orc_guo.argtypes = [_d, _dp, _dp, _dp]
    L.orc_moments.argtypes = [_dp, _dp, _vp, _dp]
    L.orc_lb_step.argtypes = [_i, _i, _i, _i, _d, _dp, _vp, _dp, _vp, _d, _vp, _d, _dp, _dp, _vp, _vp]
    L.orc_inside.argtypes = [_i, _i, _i, _i, _ip, _dp, _bp]
    L.orc_mass.argtypes = [_C.c_size_t, _dp]
    L.orc_mass.restype = _d
    L.orc_max_u.argtypes = [_C.c_size_t, _dp]
    L.orc_max_u.restype = _d
    L.orc_peskin.argtypes = [_d]
    L.orc_peskin.restype = _d
    L.orc_spread.argtypes = [_i, _i, _i, _i, _i, _dp, _dp, _dp, _dp]
    L.orc_interp.argtypes = [_i, _i, _i, _i, _dp, _i, _dp, _dp]
    L.orc_triangle_geometry.argtypes = [_i, _ip, _dp, _dp, _dp]
    L.orc_volume.argtypes = [_i, _ip, _dp]
    L.orc_volume.restype = _d
    L.orc_volume_moments.argtypes = [_i, _ip, _dp, _dp, _dp]
    L.orc_area.argtypes = [_i, _ip, _dp]
    L.orc_area.restype = _d
    L.orc_wetting_A.argtypes = [_d, _d, _d, _i, _i]
    L.orc_wetting_A.restype = _d
    L.orc_pi.argtypes = [_d, _d, _d, _i, _i]
    L.orc_pi.restype = _d
    L.orc_node_forces.argtypes = [_i, _i, _ip, _dp, _d, _d, _d, _i, _i, _d, _d,
                                  _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_node_forces.restype = _i
    L.orc_csr.argtypes = [_i, _i, _ip, _ip, _ip]
    L.orc_base_cells.argtypes = [_i, _dp, _i, _i, _ip]
    L.orc_touched_tiles.argtypes = [_i, _dp, _i, _i, _i, _i, _i, _i, _i, _bp]
    L.orc_mesh_observables.argtypes = [_i, _i, _ip, _dp, _d, _dp]


def _f64(a):
    return _np.ascontiguousarray(a, dtype=_np.float64)


def _i32(a):
    return _np.ascontiguousarray(a, dtype=_np.int32)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops from now on."""
    lib().orc_set_threads(int(n))


def lattice():
    """(c (19,3) int32, w (19,) float64, opp (19,) int32) in the oracle's order."""
    c = _np.zeros((19, 3), _np.int32)
    w = _np.zeros(19)
    o = _np.zeros(19, _np.int32)
    lib().orc_lattice(c, w, o)
    return c, w, o


def feq(rho, u):
    out = _np.zeros(19)
    lib().orc_feq(float(rho), _f64(u), out)
    return out


def guo(tau, u, F):
    out = _np.zeros(19)
    lib().orc_guo(float(tau), _f64(u), _f64(F), out)
    return out


def moments(fcell, F=(0.0, 0.0, 0.0)):
    rho = _C.c_double()
    u = _np.zeros(3)
    lib().orc_moments(_f64(fcell), _f64(F), _C.byref(rho), u)
    return rho.value, u


def peskin(r):
    return lib().orc_peskin(float(r))


def lb_step(f, tau, zbc=0, F=None, g=(0.0, 0.0, 0.0), scratch=None, want_moments=True,
            out=None, rho=None, u=None, inside=None, tau_in=0.0, u_wall=None, rho_wall=1.0):
    """One LB step.  f: (19,nz,ny,nx).  Returns (f_new, rho, u); `scratch`,
    `out`, `rho` and `u` may be passed in to reuse buffers.  `inside`
    (uint8 (nz,ny,nx)) marks the cells that relax with tau_in.  `u_wall`:
    ((ux, uy) of the wall at z = 0, (ux, uy) of the wall at z = nz), or None
    for resting walls; rho_wall enters the moving-wall term."""
    f = _f64(f)
    _, nz, ny, nx = f.shape
    fs = scratch if scratch is not None else _np.empty_like(f)
    fn = out if out is not None else _np.empty_like(f)
    if want_moments:
        rho = rho if rho is not None else _np.empty((nz, ny, nx))
        u = u if u is not None else _np.empty((3, nz, ny, nx))
    else:
        rho = u = None
    Fk = None if F is None else _f64(F)  # kept alive for the call
    ins = None if inside is None else _np.ascontiguousarray(inside, dtype=_np.uint8)
    uw = None if u_wall is None else _f64(_np.reshape(u_wall, 4))
    lib().orc_lb_step(nx, ny, nz, int(zbc), float(tau), f,
                      Fk.ctypes.data_as(_vp) if Fk is not None else None,
                      _f64(g), ins.ctypes.data_as(_vp) if ins is not None else None, float(tau_in),
                      uw.ctypes.data_as(_vp) if uw is not None else None, float(rho_wall),
                      fs, fn,
                      rho.ctypes.data_as(_vp) if rho is not None else None,
                      u.ctypes.data_as(_vp) if u is not None else None)
    return fn, rho, u


def mass(f):
    f = _f64(f)
    return lib().orc_mass(f[0].size, f)


def max_u(f):
    f = _f64(f)
    return lib().orc_max_u(f[0].size, f)


def spread(shape, zbc, q, phi, F=None):
    """Spread nodal forces phi (N,3) at q (N,3) onto a (3,nz,ny,nx) field.
    Returns (F, to_wall)."""
    nz, ny, nx = shape
    if F is None:
        F = _np.zeros((3, nz, ny, nx))
    tw = _np.zeros(3)
    lib().orc_spread(nx, ny, nz, int(zbc), len(q), _f64(q), _f64(phi), F, tw)
    return F, tw


def interp(u, zbc, q):
    u = _f64(u)
    _, nz, ny, nx = u.shape
    U = _np.zeros((len(q), 3))
    lib().orc_interp(nx, ny, nz, int(zbc), u, len(q), _f64(q), U)
    return U


def triangle_geometry(tris, q):
    T = len(tris)
    A = _np.zeros(T)
    n = _np.zeros((T, 3))
    lib().orc_triangle_geometry(T, _i32(tris), _f64(q), A, n)
    return A, n


def volume(tris, q):
    return lib().orc_volume(len(tris), _i32(tris), _f64(q))


def volume_moments(tris, q, ref=(0.0, 0.0, 0.0)):
    """(V, first moments [3], second moments [3,3]) of the enclosed volume
    about ref."""
    out = _np.zeros(10)
    lib().orc_volume_moments(len(tris), _i32(tris), _f64(q), _f64(ref), out)
    xx, yy, zz, xy, xz, yz = out[4:]
    M2 = _np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
    return out[0], out[1:4].copy(), M2


def deformation(tris, q):
    """Deformation index in the shear (x, z) plane (Sec. 4): the semi-axes
    r1 >= r3 of the ellipsoid whose second moments about the centroid equal
    the droplet's (an ellipsoid of semi-axis r along a principal direction
    has int x^2 dV = V r^2 / 5), D = (r1 - r3) / (r1 + r3); `inclination` is
    the angle of the r1 axis from the x axis toward z, in (-pi/2, pi/2]."""
    q = _f64(q)
    ref = q.mean(0)
    V, M1, M2 = volume_moments(tris, q, ref)
    c = M1 / V
    C = M2 / V - _np.outer(c, c)
    S = C[_np.ix_([0, 2], [0, 2])]
    lam, vec = _np.linalg.eigh(S)
    r3, r1 = _np.sqrt(5.0 * lam)
    v = vec[:, 1]
    ang = _np.arctan2(v[1], v[0])
    if ang <= -_np.pi / 2:
        ang += _np.pi
    elif ang > _np.pi / 2:
        ang -= _np.pi
    return {"D": (r1 - r3) / (r1 + r3), "r1": r1, "r3": r3, "inclination": ang,
            "centroid": c + ref}


def area(tris, q):
    return lib().orc_area(len(tris), _i32(tris), _f64(q))


def wetting_A(sigma, theta, xi, n=9, m=3):
    return lib().orc_wetting_A(float(sigma), float(theta), float(xi), int(n), int(m))


def pi_of_d(d, A, xi, n=9, m=3):
    return lib().orc_pi(float(d), float(A), float(xi), int(n), int(m))


def node_forces(tris, q, sigma, A, xi, n=9, m=3, k_vol=0.0, V0=1.0):
    """Returns dict with phi, phi_st, phi_pi, phi_v, chi, nhat and the count
    of nodes at or below the wall."""
    q = _f64(q)
    N = len(q)
    out = {k: _np.zeros((N, 3)) for k in ("phi", "phi_st", "phi_pi", "phi_v", "nhat")}
    out["chi"] = _np.zeros(N)
    bad = lib().orc_node_forces(N, len(tris), _i32(tris), q, float(sigma), float(A),
                                float(xi), int(n), int(m), float(k_vol), float(V0),
                                out["phi"], out["phi_st"], out["phi_pi"], out["phi_v"],
                                out["chi"], out["nhat"])
    out["below_wall"] = int(bad)
    return out


def csr(n_nodes, tris):
    off = _np.zeros(n_nodes + 1, _np.int32)
    ent = _np.zeros(3 * len(tris), _np.int32)
    lib().orc_csr(n_nodes, len(tris), _i32(tris), off, ent)
    return off, ent


def base_cells(q, nx, ny):
    b = _np.zeros((len(q), 3), _np.int32)
    lib().orc_base_cells(len(q), _f64(q), nx, ny, b)
    return b


def inside(shape, tris, q):
    """uint8 (nz,ny,nx): 1 for cells whose centre the closed mesh(es) enclose
    (parity of the crossings of the vertical ray below the centre, exact
    integer predicates)."""
    nz, ny, nx = shape
    tris = _np.ascontiguousarray(tris, dtype=_np.int32)
    out = _np.zeros((nz, ny, nx), _np.uint8)
    lib().orc_inside(nx, ny, nz, len(tris), tris, _f64(q), out)
    return out


def touched_tiles(q, shape, zbc, tile=(4, 4, 4)):
    """Flags [tiles_z][tiles_y][tiles_x] of the tiles (tile = cells per tile
    along x, y, z) that hold a cell of some node's 4x4x4 stencil."""
    nz, ny, nx = shape
    tx, ty, tz = tile
    tn = [(nz + tz - 1) // tz, (ny + ty - 1) // ty, (nx + tx - 1) // tx]
    flags = _np.zeros(tn, _np.uint8)
    lib().orc_touched_tiles(len(q), _f64(q), nx, ny, nz, int(zbc), tx, ty, tz, flags)
    return flags


def mesh_observables(tris, q, xi):
    out = _np.zeros(11)
    lib().orc_mesh_observables(len(q), len(tris), _i32(tris), _f64(q), float(xi), out)
    keys = ("volume", "area", "z_min", "z_max", "height", "cx", "cy", "cz",
            "contact_radius", "theta_app", "n_crossings")
    return dict(zip(keys, out.tolist()))


from .sim import OracleSim  # noqa: E402,F401
