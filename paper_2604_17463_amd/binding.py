"""ctypes binding of libiblb.so (include/iblb.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch provides
the device workspace and the stream."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiblb.so")

IBLB_OK = 0
IBLB_E_INVAL, IBLB_E_MESH, IBLB_E_DEVICE, IBLB_E_WORKSPACE, IBLB_E_UNSTABLE, IBLB_E_STATE = (
    -1, -2, -3, -4, -5, -6)
IBLB_F64, IBLB_F32, IBLB_F16DEV, IBLB_BF16DEV = 0, 1, 2, 3
IBLB_Z_WALLS, IBLB_Z_PERIODIC = 0, 1
IBLB_FLAG_GRAPH, IBLB_FLAG_AUTOTUNE, IBLB_FLAG_FULL_U = 1, 2, 4
IBLB_BIT_RHO, IBLB_BIT_MACH, IBLB_BIT_WALL, IBLB_BIT_JUMP, IBLB_BIT_BAND = 1, 2, 4, 8, 16

EXPORTS = (
    "iblb_velocity_set", "iblb_workspace_size", "iblb_init", "iblb_step", "iblb_step_static",
    "iblb_observables",
    "iblb_read_state", "iblb_read_window", "iblb_write_state", "iblb_read_nodes", "iblb_write_nodes",
    "iblb_compute_forces", "iblb_compute_spread", "iblb_interpolate", "iblb_read_bins",
    "iblb_read_csr", "iblb_read_inside", "iblb_state_size", "iblb_save_state", "iblb_load_state",
    "iblb_set_launch", "iblb_time_mesh_chain", "iblb_get_launch", "iblb_band_tile", "iblb_time_stream_collide",
    "iblb_destroy", "iblb_last_error",
)


class iblb_box(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("zbc", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double), ("body_force", C.c_double * 3),
                ("tau_in", C.c_double), ("wall_lo", C.c_double * 2), ("wall_hi", C.c_double * 2)]


class iblb_droplet(C.Structure):
    _fields_ = [("box", C.c_int32), ("n_nodes", C.c_int32), ("n_tris", C.c_int32),
                ("n_exp", C.c_int32), ("m_exp", C.c_int32), ("reserved", C.c_int32),
                ("nodes", C.POINTER(C.c_double)), ("tris", C.POINTER(C.c_int32)),
                ("sigma", C.c_double), ("theta_eq", C.c_double), ("xi", C.c_double),
                ("k_vol", C.c_double)]


class iblb_config(C.Structure):
    _fields_ = [("n_boxes", C.c_int32), ("n_droplets", C.c_int32),
                ("boxes", C.POINTER(iblb_box)), ("droplets", C.POINTER(iblb_droplet)),
                ("storage", C.c_int32), ("flags", C.c_uint32), ("dev_scale", C.c_double)]


class iblb_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("volume", C.c_double), ("area", C.c_double),
                ("z_min", C.c_double), ("z_max", C.c_double), ("height", C.c_double),
                ("contact_radius", C.c_double), ("theta_app", C.c_double),
                ("centroid", C.c_double * 3), ("deformation", C.c_double),
                ("inclination", C.c_double), ("n_crossings", C.c_int32),
                ("status_bits", C.c_uint32)]


class iblb_box_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("max_u", C.c_double),
                ("status_bits", C.c_uint32), ("reserved", C.c_int32)]


_lib = None


def load():
    """Load libiblb.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP/HSA runtime; loading it first makes this
    # library bind to the same runtime instead of a second copy from /opt/rocm
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2604_17463_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    L.iblb_velocity_set.argtypes = [ip, dp]
    L.iblb_workspace_size.argtypes = [C.POINTER(iblb_config), C.POINTER(C.c_size_t)]
    L.iblb_init.argtypes = [C.POINTER(iblb_config), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.iblb_step.argtypes = [vp, i64]
    L.iblb_step_static.argtypes = [vp, i64]
    L.iblb_observables.argtypes = [vp, C.POINTER(iblb_obs), i32, C.POINTER(iblb_box_obs), i32]
    L.iblb_read_state.argtypes = [vp, i32, dp, dp]
    L.iblb_read_window.argtypes = [vp, i32, ip, ip, dp, dp]
    L.iblb_write_state.argtypes = [vp, i32, dp]
    L.iblb_read_nodes.argtypes = [vp, i32, dp]
    L.iblb_write_nodes.argtypes = [vp, i32, dp]
    L.iblb_compute_forces.argtypes = [vp, i32, dp]
    L.iblb_compute_spread.argtypes = [vp, i32, dp, C.POINTER(C.c_uint8)]
    L.iblb_interpolate.argtypes = [vp, i32, dp, dp]
    L.iblb_read_bins.argtypes = [vp, i32, ip]
    L.iblb_read_csr.argtypes = [vp, i32, ip, ip]
    L.iblb_read_inside.argtypes = [vp, i32, C.POINTER(C.c_uint8)]
    L.iblb_state_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.iblb_time_mesh_chain.argtypes = [vp, i32, C.POINTER(C.c_double)]
    L.iblb_save_state.argtypes = [vp, vp, C.c_size_t]
    L.iblb_load_state.argtypes = [vp, vp, C.c_size_t]
    L.iblb_set_launch.argtypes = [vp, i32, i32, i32, i32, i32, i32]
    L.iblb_get_launch.argtypes = [vp, ip, ip, ip, ip, ip, ip]
    L.iblb_band_tile.argtypes = [ip]
    L.iblb_time_stream_collide.argtypes = [vp, i32, dp]
    L.iblb_destroy.argtypes = [vp]
    L.iblb_last_error.argtypes = [vp]
    L.iblb_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "iblb_last_error":
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


class IblbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"iblb error {code}: {msg}")
        self.code = code


def check(code, ctx=None):
    if code != IBLB_OK:
        msg = load().iblb_last_error(ctx).decode()
        raise IblbError(code, msg)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def velocity_set():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    check(load().iblb_velocity_set(_iptr(c), _dptr(w)))
    return c, w


def make_config(workload, storage=None, flags=0, dev_scale=None):
    """C structs for a workload (boxes/droplets as in iblb_inputs).  Returns
    (config, keepalive)."""
    storage = workload.storage if storage is None else storage
    dev_scale = workload.dev_scale if dev_scale is None else dev_scale
    nb, nd = len(workload.boxes), len(workload.droplets)
    boxes = (iblb_box * nb)()
    for k, b in enumerate(workload.boxes):
        boxes[k] = iblb_box(b.nx, b.ny, b.nz, b.zbc, b.tau, b.rho0,
                            (C.c_double * 3)(*[float(v) for v in b.body_force]),
                            float(getattr(b, "tau_in", 0.0)),
                            (C.c_double * 2)(*[float(v) for v in getattr(b, "wall_lo", (0.0, 0.0))]),
                            (C.c_double * 2)(*[float(v) for v in getattr(b, "wall_hi", (0.0, 0.0))]))
    drops = (iblb_droplet * max(nd, 1))()
    keep = [boxes, drops]
    for k, d in enumerate(workload.droplets):
        nodes = np.ascontiguousarray(d.nodes, dtype=np.float64)
        tris = np.ascontiguousarray(d.tris, dtype=np.int32)
        keep += [nodes, tris]
        drops[k] = iblb_droplet(d.box, len(nodes), len(tris), d.n_exp, d.m_exp, 0,
                                _dptr(nodes), _iptr(tris), d.sigma, d.theta_eq, d.xi, d.k_vol)
    cfg = iblb_config(nb, nd, boxes, drops if nd else None, storage, flags, float(dev_scale))
    return cfg, keep


def band_tile():
    """(x, y, z) cells of the band tiles that compute_spread's flags refer to."""
    shape = (C.c_int32 * 3)()
    check(load().iblb_band_tile(shape))
    return tuple(shape)


def workspace_size(cfg) -> int:
    n = C.c_size_t()
    check(load().iblb_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


class Simulation:
    """One library context over a workload, with its workspace in a torch
    uint8 tensor on the current device and all work on torch's current
    stream."""

    def __init__(self, workload, storage=None, flags=0, dev_scale=None, device="cuda"):
        import torch

        self._torch = torch
        self.wl = workload
        self.cfg, self._keep = make_config(workload, storage, flags, dev_scale)
        self.bytes = workspace_size(self.cfg)
        self.ws = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.ws.device)
        ctx = C.c_void_p()
        check(load().iblb_init(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()),
                               self.bytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.nb, self.nd = len(workload.boxes), len(workload.droplets)

    def close(self):
        if self.ctx:
            load().iblb_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code):
        check(code, self.ctx)

    def step(self, n=1):
        self._chk(load().iblb_step(self.ctx, int(n)))

    def step_static(self, n=1):
        """The same steps, with the step scratch in the library's fixed
        device array (no allocation)."""
        self._chk(load().iblb_step_static(self.ctx, int(n)))

    def observables(self, raise_unstable=True):
        drops = (iblb_obs * max(self.nd, 1))()
        boxes = (iblb_box_obs * self.nb)()
        code = load().iblb_observables(self.ctx, drops if self.nd else None, self.nd, boxes, self.nb)
        if code != IBLB_OK and (raise_unstable or code != IBLB_E_UNSTABLE):
            self._chk(code)
        out_d = []
        for k in range(self.nd):
            o = drops[k]
            out_d.append({"step": o.step, "volume": o.volume, "area": o.area, "z_min": o.z_min,
                          "z_max": o.z_max, "height": o.height, "contact_radius": o.contact_radius,
                          "theta_app": o.theta_app, "cx": o.centroid[0], "cy": o.centroid[1],
                          "cz": o.centroid[2], "n_crossings": o.n_crossings,
                          "deformation": o.deformation, "inclination": o.inclination,
                          "status_bits": o.status_bits})
        out_b = [{"step": b.step, "mass": b.mass, "max_u": b.max_u, "status_bits": b.status_bits}
                 for b in boxes]
        return out_d, out_b

    def _box(self, b):
        bx = self.wl.boxes[b]
        return bx.nz, bx.ny, bx.nx

    def read_state(self, b=0, want_u=False):
        nz, ny, nx = self._box(b)
        f = np.empty((19, nz, ny, nx))
        u = np.empty((3, nz, ny, nx)) if want_u else None
        self._chk(load().iblb_read_state(self.ctx, b, _dptr(f), _dptr(u) if want_u else None))
        return (f, u) if want_u else f

    def read_window(self, lo, ext, b=0, want_u=False):
        """Populations (and velocity) of the cells lo + [0, ext) of box b,
        periodic sides wrapped; f [19][ez][ey][ex]."""
        lo3 = (C.c_int32 * 3)(*[int(v) for v in lo])
        ext3 = (C.c_int32 * 3)(*[int(v) for v in ext])
        ex, ey, ez = (int(v) for v in ext)
        f = np.empty((19, ez, ey, ex))
        u = np.empty((3, ez, ey, ex)) if want_u else None
        self._chk(load().iblb_read_window(self.ctx, b, lo3, ext3, _dptr(f), _dptr(u) if want_u else None))
        return (f, u) if want_u else f

    def write_state(self, f, b=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._chk(load().iblb_write_state(self.ctx, b, _dptr(f)))

    def read_nodes(self, d=0):
        q = np.empty((len(self.wl.droplets[d].nodes), 3))
        self._chk(load().iblb_read_nodes(self.ctx, d, _dptr(q)))
        return q

    def write_nodes(self, q, d=0):
        q = np.ascontiguousarray(q, dtype=np.float64)
        self._chk(load().iblb_write_nodes(self.ctx, d, _dptr(q)))

    def compute_forces(self, d=0):
        phi = np.empty((len(self.wl.droplets[d].nodes), 3))
        self._chk(load().iblb_compute_forces(self.ctx, d, _dptr(phi)))
        return phi

    def compute_spread(self, b=0, want_F=True):
        """Spread force density of box b ([3][nz][ny][nx], or None without
        want_F) and the flags of the band tiles holding a stencil cell."""
        nz, ny, nx = self._box(b)
        F = np.empty((3, nz, ny, nx)) if want_F else None
        tx, ty, tz = band_tile()
        flags = np.zeros((-(-nz // tz), -(-ny // ty), -(-nx // tx)), np.uint8)
        self._chk(load().iblb_compute_spread(self.ctx, b, _dptr(F) if want_F else None,
                                             flags.ctypes.data_as(C.POINTER(C.c_uint8))))
        return F, flags

    def interpolate(self, u, d=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        U = np.empty((len(self.wl.droplets[d].nodes), 3))
        self._chk(load().iblb_interpolate(self.ctx, d, _dptr(u), _dptr(U)))
        return U

    def read_bins(self, d=0):
        b = np.empty((len(self.wl.droplets[d].nodes), 3), np.int32)
        self._chk(load().iblb_read_bins(self.ctx, d, _iptr(b)))
        return b

    def read_csr(self, d=0):
        dr = self.wl.droplets[d]
        off = np.empty(len(dr.nodes) + 1, np.int32)
        ent = np.empty(3 * len(dr.tris), np.int32)
        self._chk(load().iblb_read_csr(self.ctx, d, _iptr(off), _iptr(ent)))
        return off, ent

    def save_state(self):
        """The whole state of the current time as bytes (iblb_save_state)."""
        n = C.c_size_t()
        self._chk(load().iblb_state_size(self.ctx, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._chk(load().iblb_save_state(self.ctx, buf, n.value))
        return bytes(buf)

    def load_state(self, blob):
        """Restore a state saved from a context of the same configuration."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._chk(load().iblb_load_state(self.ctx, buf, len(blob)))

    def read_inside(self, b=0):
        """Inside bits of box b at the current node positions, uint8 [nz][ny][nx]."""
        bx = self.wl.boxes[b]
        m = np.empty((bx.nz, bx.ny, bx.nx), np.uint8)
        self._chk(load().iblb_read_inside(self.ctx, b, m.ctypes.data_as(C.POINTER(C.c_uint8))))
        return m

    def set_launch(self, threads_x, rows, cells_per_thread=1, streaming_stores=0, max_workgroups=0,
                   band_after_bulk=0):
        self._chk(load().iblb_set_launch(self.ctx, int(threads_x), int(rows), int(cells_per_thread),
                                         int(streaming_stores), int(max_workgroups),
                                         int(band_after_bulk)))

    def get_launch(self):
        """(threads_x, rows_per_group, cells_per_thread, streaming_stores,
        max_workgroups, band_after_bulk) of the bulk kernel and the step."""
        v = [C.c_int32() for _ in range(6)]
        self._chk(load().iblb_get_launch(self.ctx, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def time_stream_collide(self, reps=10):
        ms = C.c_double()
        self._chk(load().iblb_time_stream_collide(self.ctx, int(reps), C.byref(ms)))
        return ms.value

    def time_mesh_chain(self, reps=10):
        ms = C.c_double()
        self._chk(load().iblb_time_mesh_chain(self.ctx, int(reps), C.byref(ms)))
        return ms.value
