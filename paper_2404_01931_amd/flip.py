"""Thin ctypes binding of libflipmi (include/flip.h): argument marshalling only.

Every step of the FLIP timestep runs in the HIP kernels of libflipmi.so; this
module allocates the device workspace and passes streams through PyTorch, and
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; FLIPMI_LIB names another build of the same library
LIB_PATH = os.environ.get("FLIPMI_LIB") or os.path.join(_PKG, "libflipmi.so")

FLIP_OK = 0
FLIP_E_INVALID = -1
FLIP_E_WORKSPACE = -2
FLIP_E_HIP = -3
FLIP_E_NOT_CONVERGED = -4
FLIP_E_NONFINITE = -5
FLIP_E_STATE = -6

FLIP_FP32, FLIP_FP64, FLIP_MIXED = 0, 1, 2
FLIP_REGION_BOX, FLIP_REGION_SPHERE = 0, 1

FLIP_FLAG_NO_GRAVITY = 1
FLIP_FLAG_NO_PROJECTION = 2
FLIP_FLAG_ADVECT_PARTICLE_VEL = 4
FLIP_FLAG_KERNEL_TIMING = 8
FLIP_FLAG_MULTIGRID = 16
FLIP_FLAG_RED_BLACK_GS = 32
FLIP_FLAG_ADAPTIVE_DT = 64
FLIP_FLAG_RESEED = 128
FLIP_FLAG_DIAGNOSTICS = 256

FLIP_FIELD_POS = 0
FLIP_FIELD_VEL = 1
FLIP_FIELD_ID = 2
FLIP_FIELD_CELL_COUNT = 3
FLIP_FIELD_CELL_START = 4
FLIP_FIELD_FLAGS = 5
FLIP_FIELD_U_OLD = 6
FLIP_FIELD_U_STAR = 7
FLIP_FIELD_U_NEW = 8
FLIP_FIELD_RHS = 9
FLIP_FIELD_PRESSURE = 10
FLIP_FIELD_DIV = 11

KERNEL_NAMES = ["bin_keys", "bin_scan", "bin_scatter", "bin_gather", "tiles", "p2g", "rhs",
                "pcg_direction", "pcg_update", "project", "g2p", "mg_down_fine", "mg_up_fine",
                "mg_coarse"]
FLIP_KERNEL_COUNT = len(KERNEL_NAMES)

FLIP_BATCH_MAX_SCENES = 256
FLIP_BATCH_GRAPHS = 1
FLIP_BATCH_MULTIGRID = 2

EXPORTED = ["flip_workspace_bytes", "flip_init", "flip_step", "flip_field_bytes", "flip_readback",
            "flip_stats", "flip_destroy", "flip_status_string", "flip_batch_workspace_bytes",
            "flip_batch_create", "flip_batch_step", "flip_batch_destroy", "flip_surface_field_bytes",
            "flip_surface_field", "flip_surface_mesh_workspace_bytes", "flip_surface_mesh",
            "flip_surface_mesh_noalloc", "flip_batch_slots_workspace_bytes", "flip_batch_create_slots",
            "flip_batch_attach", "flip_batch_detach", "flip_batch_get_info"]

# device scratch of flip_surface_mesh_noalloc per GPU (FLIP_MESH_SCRATCH_MAX_BYTES)
FLIP_MESH_SCRATCH_MAX_BYTES = 64 << 20


class FlipError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


class flip_region(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("center", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("vel", ctypes.c_double * 3)]


class flip_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("flip_ratio", ctypes.c_double), ("density", ctypes.c_double),
                ("pcg_tol", ctypes.c_double), ("pcg_max_iters", ctypes.c_int32),
                ("ir_tol", ctypes.c_double), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("n_regions", ctypes.c_uint32), ("regions", ctypes.POINTER(flip_region)),
                ("subcells_per_axis", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("n_particles", ctypes.c_int64), ("pos0", ctypes.POINTER(ctypes.c_double)),
                ("vel0", ctypes.POINTER(ctypes.c_double)), ("cfl", ctypes.c_double),
                ("particle_capacity", ctypes.c_int64)]


class flip_step_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("n_particles", ctypes.c_int64),
                ("n_fluid_cells", ctypes.c_int64), ("n_active_tiles", ctypes.c_int64),
                ("pcg_iterations", ctypes.c_int32), ("pcg_status", ctypes.c_int32),
                ("max_b", ctypes.c_double), ("max_r", ctypes.c_double),
                ("pcg_iterations_total", ctypes.c_int64), ("pcg_cell_iterations_total", ctypes.c_int64),
                ("latched_status", ctypes.c_int32), ("refinements", ctypes.c_int32), ("kernel_ms", ctypes.c_double * FLIP_KERNEL_COUNT),
                ("kernel_launches", ctypes.c_int64 * FLIP_KERNEL_COUNT), ("dt", ctypes.c_double),
                ("n_reseeded", ctypes.c_int64), ("true_residual", ctypes.c_double),
                ("div_ratio", ctypes.c_double), ("kinetic_energy", ctypes.c_double),
                ("max_speed", ctypes.c_double), ("cfl_number", ctypes.c_double),
                ("nonfinite", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class flip_batch_slots(ctypes.Structure):
    _fields_ = [("nslots", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_nx", ctypes.c_int32), ("max_ny", ctypes.c_int32), ("max_nz", ctypes.c_int32)]


class flip_batch_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64), ("table_uploads", ctypes.c_int64),
                ("nslots", ctypes.c_int32), ("occupied", ctypes.c_int32)]


_lib = None


def load():
    """Load libflipmi.so; raises if it is missing (no fallback of any kind)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2404_01931_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        cfgp = ctypes.POINTER(flip_config)
        lib.flip_workspace_bytes.argtypes = [cfgp, ctypes.POINTER(sz)]
        lib.flip_init.argtypes = [cfgp, vp, sz, vp, ctypes.POINTER(vp)]
        lib.flip_step.argtypes = [vp, i32, vp]
        lib.flip_field_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        lib.flip_readback.argtypes = [vp, i32, vp, sz, i32, vp]
        lib.flip_stats.argtypes = [vp, ctypes.POINTER(flip_step_stats)]
        lib.flip_destroy.argtypes = [vp]
        lib.flip_destroy.restype = None
        lib.flip_status_string.argtypes = [i32]
        lib.flip_status_string.restype = ctypes.c_char_p
        vpp = ctypes.POINTER(vp)
        lib.flip_batch_workspace_bytes.argtypes = [vpp, i32, ctypes.POINTER(sz)]
        lib.flip_batch_create.argtypes = [vpp, i32, ctypes.c_uint32, vp, sz, vp, vpp]
        lib.flip_batch_step.argtypes = [vp, i32, vp]
        lib.flip_batch_destroy.argtypes = [vp]
        lib.flip_batch_destroy.restype = None
        lib.flip_surface_field_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        lib.flip_surface_field.argtypes = [vp, ctypes.c_double, ctypes.c_double, i32, vp, sz, vp]
        lib.flip_surface_mesh_workspace_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.flip_surface_mesh.argtypes = [vp, vp, i32, vp, sz, vp, vp, ctypes.c_int64, vp, ctypes.c_int64, i64p,
                                          i64p, vp]
        lib.flip_surface_mesh_noalloc.argtypes = [vp, vp, i32, vp, vp, ctypes.c_int64, vp, ctypes.c_int64, i64p,
                                                  i64p, vp]
        specp = ctypes.POINTER(flip_batch_slots)
        lib.flip_batch_slots_workspace_bytes.argtypes = [specp, ctypes.POINTER(sz)]
        lib.flip_batch_create_slots.argtypes = [specp, vp, sz, vp, vpp]
        lib.flip_batch_attach.argtypes = [vp, i32, vp]
        lib.flip_batch_detach.argtypes = [vp, i32]
        lib.flip_batch_get_info.argtypes = [vp, ctypes.POINTER(flip_batch_info)]
        for name in ["flip_workspace_bytes", "flip_init", "flip_step", "flip_field_bytes",
                     "flip_readback", "flip_stats", "flip_batch_workspace_bytes", "flip_batch_create",
                     "flip_batch_step", "flip_surface_field_bytes", "flip_surface_field",
                     "flip_surface_mesh_workspace_bytes", "flip_surface_mesh", "flip_surface_mesh_noalloc",
                     "flip_batch_slots_workspace_bytes", "flip_batch_create_slots", "flip_batch_attach",
                     "flip_batch_detach", "flip_batch_get_info"]:
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().flip_status_string(int(status)).decode()


def _check(status: int, where: str, allow=()):
    if status != FLIP_OK and status not in allow:
        raise FlipError(status, where)
    return status


# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------

def make_config(shape, dx, dt, *, gravity=(0.0, -9.81, 0.0), flip_ratio=0.95, density=1.0,
                pcg_tol=1e-6, pcg_max_iters=0, ir_tol=1e-8, precision=FLIP_FP32, flags=0,
                regions=(), subcells=2, seed=0, pos0=None, vel0=None, cfl=0.0, capacity=0):
    """Build a flip_config. Returns (config, keepalive) - keep both alive while in use."""
    cfg = flip_config()
    cfg.nx, cfg.ny, cfg.nz = (int(v) for v in shape)
    cfg.dx = float(dx)
    cfg.gravity[:] = [float(g) for g in gravity]
    cfg.dt = float(dt)
    cfg.flip_ratio = float(flip_ratio)
    cfg.density = float(density)
    cfg.pcg_tol = float(pcg_tol)
    cfg.pcg_max_iters = int(pcg_max_iters)
    cfg.ir_tol = float(ir_tol)
    cfg.precision = int(precision)
    cfg.flags = int(flags)
    cfg.cfl = float(cfl)
    cfg.particle_capacity = int(capacity)
    keep = []
    if pos0 is not None:
        p = np.ascontiguousarray(pos0, dtype=np.float64).reshape(3, -1)
        v = np.ascontiguousarray(vel0, dtype=np.float64).reshape(3, -1)
        assert p.shape == v.shape
        keep += [p, v]
        cfg.n_particles = p.shape[1]
        cfg.pos0 = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.vel0 = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    else:
        arr = (flip_region * max(1, len(regions)))()
        for t, r in enumerate(regions):
            arr[t].kind = FLIP_REGION_BOX if r.kind == "box" else FLIP_REGION_SPHERE
            arr[t].lo[:] = [float(q) for q in r.lo]
            arr[t].hi[:] = [float(q) for q in r.hi]
            arr[t].center[:] = [float(q) for q in r.center]
            arr[t].radius = float(r.radius)
            arr[t].vel[:] = [float(q) for q in r.vel]
        keep.append(arr)
        cfg.n_regions = len(regions)
        cfg.regions = arr
    # the seeding density and jitter also drive reseeding
    cfg.subcells_per_axis = int(subcells)
    cfg.seed = int(seed)
    return cfg, keep


def scene_config(sc, *, precision=None, flags=0, pcg_tol=None, pcg_max_iters=0, pos0=None, vel0=None, cfl=0.0,
                 capacity=0):
    """flip_config for a scene of ``paper_2404_01931_amd.inputs``."""
    prec = {"fp32": FLIP_FP32, "fp64": FLIP_FP64, "mixed": FLIP_MIXED}[sc.precision]
    if precision is not None:
        prec = precision
    return make_config((sc.n, sc.n, sc.n), sc.dx, sc.dt, gravity=sc.gravity, flip_ratio=sc.flip_ratio,
                       density=sc.density, pcg_tol=sc.tol if pcg_tol is None else pcg_tol,
                       pcg_max_iters=pcg_max_iters, ir_tol=sc.ir_tol, precision=prec, flags=flags,
                       regions=sc.regions, subcells=sc.sub, seed=sc.seed, pos0=pos0, vel0=vel0, cfl=cfl,
                       capacity=capacity)


# --------------------------------------------------------------------------
# the C ABI, one function per entry point
# --------------------------------------------------------------------------

def flip_workspace_bytes(cfg: flip_config) -> int:
    out = ctypes.c_size_t(0)
    _check(load().flip_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "flip_workspace_bytes")
    return out.value


def flip_init(cfg: flip_config, ws_ptr: int, ws_bytes: int, stream: int):
    h = ctypes.c_void_p(0)
    _check(load().flip_init(ctypes.byref(cfg), ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream),
                            ctypes.byref(h)), "flip_init")
    return h


def flip_step(h, nsteps: int, stream: int, allow=()) -> int:
    return _check(load().flip_step(h, int(nsteps), ctypes.c_void_p(stream)), "flip_step", allow)


def flip_field_bytes(h, field: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().flip_field_bytes(h, int(field), ctypes.byref(out)), "flip_field_bytes")
    return out.value


def flip_readback(h, field: int, dst_ptr: int, dst_bytes: int, dst_is_device: bool, stream: int):
    _check(load().flip_readback(h, int(field), ctypes.c_void_p(dst_ptr), int(dst_bytes),
                                1 if dst_is_device else 0, ctypes.c_void_p(stream)), "flip_readback")


def flip_stats(h) -> flip_step_stats:
    st = flip_step_stats()
    _check(load().flip_stats(h, ctypes.byref(st)), "flip_stats")
    return st


def flip_destroy(h):
    load().flip_destroy(h)


def _handle_array(handles):
    arr = (ctypes.c_void_p * max(1, len(handles)))()
    for i, h in enumerate(handles):
        arr[i] = h.value if isinstance(h, ctypes.c_void_p) else h
    return arr


def flip_batch_workspace_bytes(handles) -> int:
    out = ctypes.c_size_t(0)
    arr = _handle_array(handles)
    _check(load().flip_batch_workspace_bytes(arr, len(handles), ctypes.byref(out)),
           "flip_batch_workspace_bytes")
    return out.value


def flip_batch_create(handles, flags: int, ws_ptr: int, ws_bytes: int, stream: int):
    b = ctypes.c_void_p(0)
    arr = _handle_array(handles)
    _check(load().flip_batch_create(arr, len(handles), int(flags), ctypes.c_void_p(ws_ptr), ws_bytes,
                                    ctypes.c_void_p(stream), ctypes.byref(b)), "flip_batch_create")
    return b


def flip_batch_step(b, nsteps: int, stream: int, allow=()) -> int:
    return _check(load().flip_batch_step(b, int(nsteps), ctypes.c_void_p(stream)), "flip_batch_step", allow)


def flip_batch_destroy(b):
    load().flip_batch_destroy(b)


def flip_batch_slots_workspace_bytes(spec: flip_batch_slots) -> int:
    out = ctypes.c_size_t(0)
    _check(load().flip_batch_slots_workspace_bytes(ctypes.byref(spec), ctypes.byref(out)),
           "flip_batch_slots_workspace_bytes")
    return out.value


def flip_batch_create_slots(spec: flip_batch_slots, ws_ptr: int, ws_bytes: int, stream: int):
    b = ctypes.c_void_p(0)
    _check(load().flip_batch_create_slots(ctypes.byref(spec), ctypes.c_void_p(ws_ptr), ws_bytes,
                                          ctypes.c_void_p(stream), ctypes.byref(b)), "flip_batch_create_slots")
    return b


def flip_batch_attach(b, slot: int, h):
    _check(load().flip_batch_attach(b, int(slot), h), "flip_batch_attach")


def flip_batch_detach(b, slot: int):
    _check(load().flip_batch_detach(b, int(slot)), "flip_batch_detach")


def flip_batch_get_info(b) -> flip_batch_info:
    out = flip_batch_info()
    _check(load().flip_batch_get_info(b, ctypes.byref(out)), "flip_batch_get_info")
    return out


# --------------------------------------------------------------------------
# convenience wrapper used by the tests and the benchmark
# --------------------------------------------------------------------------

class Simulation:
    """A handle plus its torch-allocated device workspace, on one stream."""

    def __init__(self, cfg: flip_config, keep=None, device: str = "cuda", stream=None):
        import torch

        self._keep = keep
        self.cfg = cfg
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws_bytes = flip_workspace_bytes(cfg)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.h = flip_init(cfg, self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        self.real = np.float64 if cfg.precision == FLIP_FP64 else np.float32
        self.shape = (cfg.nx, cfg.ny, cfg.nz)

    @property
    def n(self) -> int:
        return int(self.stats().n_particles)

    def step(self, nsteps: int = 1, allow=()):
        return flip_step(self.h, nsteps, self.stream.cuda_stream, allow)

    def stats(self) -> flip_step_stats:
        return flip_stats(self.h)

    def _dtype(self, field):
        if field in (FLIP_FIELD_ID, FLIP_FIELD_CELL_COUNT, FLIP_FIELD_CELL_START):
            return np.uint32
        if field == FLIP_FIELD_FLAGS:
            return np.uint8
        if field in (FLIP_FIELD_RHS, FLIP_FIELD_PRESSURE) and self.cfg.precision == FLIP_MIXED:
            return np.float64
        if field == FLIP_FIELD_DIV:
            return np.float64
        return self.real

    def read(self, field: int) -> np.ndarray:
        nbytes = flip_field_bytes(self.h, field)
        out = np.empty(nbytes // np.dtype(self._dtype(field)).itemsize, dtype=self._dtype(field))
        flip_readback(self.h, field, out.ctypes.data, nbytes, False, self.stream.cuda_stream)
        if field in (FLIP_FIELD_POS, FLIP_FIELD_VEL):
            out = out.reshape(3, -1)
        return out

    def surface_field_device(self, radius: float, search: float, refine: int = 1):
        """Surface scalar field (Sec. 3.3.1) into a new device tensor of shape
        (nz*refine+1, ny*refine+1, nx*refine+1), stream-ordered."""
        nbytes = ctypes.c_size_t(0)
        _check(load().flip_surface_field_bytes(self.h, int(refine), ctypes.byref(nbytes)),
               "flip_surface_field_bytes")
        c = self.cfg
        shape = (c.nz * refine + 1, c.ny * refine + 1, c.nx * refine + 1)
        dt = self.torch.float64 if c.precision == FLIP_FP64 else self.torch.float32
        phi = self.torch.empty(shape, dtype=dt, device=self.ws.device)
        assert phi.numel() * phi.element_size() == nbytes.value
        _check(load().flip_surface_field(self.h, float(radius), float(search), int(refine),
                                         ctypes.c_void_p(phi.data_ptr()), nbytes.value,
                                         ctypes.c_void_p(self.stream.cuda_stream)), "flip_surface_field")
        return phi

    def surface_field(self, radius: float, search: float, refine: int = 1) -> np.ndarray:
        """Surface scalar field (Sec. 3.3.1) as a host array (synchronises)."""
        phi = self.surface_field_device(radius, search, refine)
        self.stream.synchronize()
        return phi.cpu().numpy()

    def surface_mesh_device(self, phi, refine: int = 1):
        """Marching cubes (Sec. 3.3.2) of a device corner field from
        surface_field_device: (vertices (nv, 3), normals (nv, 3), triangles
        (nt, 3) int32) as device tensors."""
        lib = load()
        wb = ctypes.c_size_t(0)
        _check(lib.flip_surface_mesh_workspace_bytes(self.h, int(refine), ctypes.byref(wb)),
               "flip_surface_mesh_workspace_bytes")
        if getattr(self, "_mc_work", None) is None or self._mc_work.numel() < wb.value:
            self._mc_work = self.torch.empty(wb.value, dtype=self.torch.uint8, device=self.ws.device)
        work = ctypes.c_void_p(self._mc_work.data_ptr())
        st = ctypes.c_void_p(self.stream.cuda_stream)
        nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
        null = ctypes.c_void_p(0)
        _check(lib.flip_surface_mesh(self.h, ctypes.c_void_p(phi.data_ptr()), int(refine), work, wb.value, null,
                                     null, 0, null, 0, ctypes.byref(nv), ctypes.byref(nt), st),
               "flip_surface_mesh (count)")
        verts = self.torch.empty((nv.value, 3), dtype=phi.dtype, device=self.ws.device)
        normals = self.torch.empty((nv.value, 3), dtype=phi.dtype, device=self.ws.device)
        tris = self.torch.empty((nt.value, 3), dtype=self.torch.int32, device=self.ws.device)
        _check(lib.flip_surface_mesh(self.h, ctypes.c_void_p(phi.data_ptr()), int(refine), work, wb.value,
                                     ctypes.c_void_p(verts.data_ptr()), ctypes.c_void_p(normals.data_ptr()),
                                     nv.value, ctypes.c_void_p(tris.data_ptr()), nt.value, ctypes.byref(nv),
                                     ctypes.byref(nt), st), "flip_surface_mesh")
        return verts, normals, tris

    def surface_mesh_noalloc_device(self, phi, refine: int = 1, out=None):
        """Marching cubes through flip_surface_mesh_noalloc (the library's own
        device scratch instead of a workspace). With out = (vertices, normals,
        triangles) preallocated device tensors the call writes into them and
        returns them cut to the mesh's size; without, it counts first and
        allocates the outputs here (the library call itself allocates nothing)."""
        lib = load()
        st = ctypes.c_void_p(self.stream.cuda_stream)
        nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
        null = ctypes.c_void_p(0)
        if out is None:
            _check(lib.flip_surface_mesh_noalloc(self.h, ctypes.c_void_p(phi.data_ptr()), int(refine), null, null, 0,
                                                 null, 0, ctypes.byref(nv), ctypes.byref(nt), st),
                   "flip_surface_mesh_noalloc (count)")
            out = (self.torch.empty((nv.value, 3), dtype=phi.dtype, device=self.ws.device),
                   self.torch.empty((nv.value, 3), dtype=phi.dtype, device=self.ws.device),
                   self.torch.empty((nt.value, 3), dtype=self.torch.int32, device=self.ws.device))
        verts, normals, tris = out
        _check(lib.flip_surface_mesh_noalloc(self.h, ctypes.c_void_p(phi.data_ptr()), int(refine),
                                             ctypes.c_void_p(verts.data_ptr()), ctypes.c_void_p(normals.data_ptr()),
                                             verts.shape[0], ctypes.c_void_p(tris.data_ptr()), tris.shape[0],
                                             ctypes.byref(nv), ctypes.byref(nt), st), "flip_surface_mesh_noalloc")
        return verts[:nv.value], normals[:nv.value], tris[:nt.value]

    def read_device(self, field: int):
        """Stream-ordered device-to-device readback into a new torch tensor of bytes."""
        nbytes = flip_field_bytes(self.h, field)
        t = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.ws.device)
        flip_readback(self.h, field, t.data_ptr(), nbytes, True, self.stream.cuda_stream)
        return t

    def faces(self, field: int):
        """Split a face field into its (u, v, w) flat arrays."""
        f = self.read(field)
        nx, ny, nz = self.shape
        sizes = [(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)]
        return [f[:sizes[0]], f[sizes[0]:sizes[0] + sizes[1]], f[sizes[0] + sizes[1]:]]

    def close(self):
        if self.h is not None:
            flip_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlotBatch:
    """A slot batch (continuous batching) plus its torch-allocated table workspace:
    Simulations join with attach() and leave with detach() between steps."""

    def __init__(self, nslots: int, precision: int = FLIP_FP32, multigrid: bool = False, graphs: bool = True,
                 max_dims=(96, 96, 96), stream=None, device: str = "cuda"):
        import torch

        self.stream = stream if stream is not None else torch.cuda.current_stream()
        flags = (FLIP_BATCH_GRAPHS if graphs else 0) | (FLIP_BATCH_MULTIGRID if multigrid else 0)
        self.spec = flip_batch_slots(int(nslots), int(precision), flags, *[int(d) for d in max_dims])
        self.ws_bytes = flip_batch_slots_workspace_bytes(self.spec)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.b = flip_batch_create_slots(self.spec, ptr, self.ws_bytes, self.stream.cuda_stream)
        self.sims = [None] * int(nslots)

    def attach(self, slot: int, sim):
        flip_batch_attach(self.b, slot, sim.h)
        self.sims[slot] = sim

    def detach(self, slot: int):
        flip_batch_detach(self.b, slot)
        self.sims[slot] = None

    def free_slot(self) -> int:
        return self.sims.index(None)

    def step(self, nsteps: int = 1, allow=()):
        return flip_batch_step(self.b, nsteps, self.stream.cuda_stream, allow)

    def info(self) -> flip_batch_info:
        return flip_batch_get_info(self.b)

    def close(self):
        if self.b is not None:
            flip_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch over several Simulations plus its torch-allocated table workspace."""

    def __init__(self, sims, flags: int = 0, stream=None):
        import torch

        self.sims = list(sims)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handles = [s.h for s in self.sims]
        self.ws_bytes = flip_batch_workspace_bytes(handles)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.sims[0].ws.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.b = flip_batch_create(handles, flags, ptr, self.ws_bytes, self.stream.cuda_stream)

    def step(self, nsteps: int = 1, allow=()):
        return flip_batch_step(self.b, nsteps, self.stream.cuda_stream, allow)

    def close(self):
        if self.b is not None:
            flip_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
