"""FP64 CPU oracle for one FLIP timestep (arXiv 2404.01931).

TEST INFRASTRUCTURE ONLY. The slow, plain reference the GPU library is checked
against. Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it. It shares no code with the GPU library and
the library never calls it.

The arithmetic lives in ``flip_oracle.c`` (plain C, double precision); this
module only marshals numpy arrays and composes the stages of one step in the
order the paper's splitting fixes (Sec. 2.1.3: force, advect, project; with the
particle stages of Sec. 3.1.3-3.1.8):

    bin -> particle-to-grid -> gravity + walls -> right-hand side
        -> PCG solve -> projection -> grid-to-particle + advection

The dense solve used as a pin in the tests is numpy's, not this module's.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flip_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

PRECOND_MIC0 = 0
PRECOND_JACOBI = 1
ADVECT_PARTICLE_VEL = 4

STATUS_CONVERGED = 0
STATUS_MAX_ITERS = 1
STATUS_BREAKDOWN = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liborc.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", _LIB, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double)]


class _Region(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("center", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("vel", ctypes.c_double * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        G = ctypes.POINTER(_Grid)
        i64, i32, dbl, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        sig = {
            "orc_face_count": (i64, [G, i32]),
            "orc_uniform01": (dbl, [u64, u64]),
            "orc_seed": (i64, [G, ctypes.POINTER(_Region), i32, i32, u64, P, P, P, P, P, P]),
            "orc_cell_keys": (None, [G, i64, P, P, P, P]),
            "orc_bin": (None, [G, i64, P, P, P, P, P, P, P]),
            "orc_fluid_flags": (None, [G, P, P]),
            "orc_p2g": (None, [G, i32, i64, P, P, P, P, P, P]),
            "orc_forces_walls": (None, [G, i32, dbl, dbl, P]),
            "orc_divergence": (None, [G, P, P, P, P]),
            "orc_rhs": (None, [G, P, P, P, P, dbl, dbl, P]),
            "orc_apply_A": (None, [G, P, P, P]),
            "orc_pcg": (i32, [G, P, P, P, dbl, i32, i32, P, P, P]),
            "orc_project": (None, [G, i32, P, P, dbl, dbl, P, P]),
            "orc_interp": (dbl, [G, i32, P, dbl, dbl, dbl]),
            "orc_g2p_advect": (None, [G, i64, P, P, P, P, P, P, P, P, dbl, dbl, ctypes.c_uint]),
            "orc_cfl_dt": (dbl, [i64, P, P, P, dbl, dbl, dbl]),
            "orc_reseed": (i64, [G, i32, u64, i64, i32, P, P, P, P, P, P, P, P, P, P, P, P]),
            "orc_surface_field": (None, [G, i32, dbl, dbl, i64, P, P, P, P]),
            "orc_surface_mesh": (i64, [G, i32, P, P, P, P, ctypes.POINTER(i64)]),
            "orc_mc_case_triangles": (i32, [ctypes.c_uint, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def face_shape(self, a: int):
        d = [self.nx, self.ny, self.nz]
        d[a] += 1
        return (d[2], d[1], d[0])

    def nfaces(self, a: int):
        s = self.face_shape(a)
        return s[0] * s[1] * s[2]

    def c(self):
        return ctypes.byref(_Grid(self.nx, self.ny, self.nz, float(self.dx)))


@dataclass
class Region:
    kind: str  # "box" or "sphere"
    lo: tuple = (-np.inf, -np.inf, -np.inf)
    hi: tuple = (np.inf, np.inf, np.inf)
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    vel: tuple = (0.0, 0.0, 0.0)


def _regions(regions):
    arr = (_Region * max(1, len(regions)))()
    for t, r in enumerate(regions):
        arr[t].kind = 0 if r.kind == "box" else 1
        for a in range(3):
            arr[t].lo[a] = r.lo[a]
            arr[t].hi[a] = r.hi[a]
            arr[t].center[a] = r.center[a]
            arr[t].vel[a] = r.vel[a]
        arr[t].radius = r.radius
    return arr


def uniform01(seed: int, counter: int) -> float:
    return _load().orc_uniform01(seed, counter)


def seed(grid: Grid, regions, sub: int, seed_value: int):
    """Jittered seeding (paper Sec. 3.1.2). Returns pos (3, n) and vel (3, n)."""
    lib = _load()
    regs = _regions(regions)
    n = lib.orc_seed(grid.c(), regs, len(regions), sub, seed_value, None, None, None, None, None, None)
    pos = np.zeros((3, n), np.float64)
    vel = np.zeros((3, n), np.float64)
    lib.orc_seed(grid.c(), regs, len(regions), sub, seed_value,
                 _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(vel[0]), _ptr(vel[1]), _ptr(vel[2]))
    return pos, vel


def cell_keys(grid: Grid, pos) -> np.ndarray:
    pos = _f64(pos)
    n = pos.shape[1]
    key = np.zeros(n, np.uint32)
    _load().orc_cell_keys(grid.c(), n, _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(key))
    return key


def bin_particles(grid: Grid, pos):
    """Binning (paper Sec. 3.1.5): key, count, start (exclusive scan), perm."""
    pos = _f64(pos)
    n = pos.shape[1]
    key = np.zeros(n, np.uint32)
    count = np.zeros(grid.ncells, np.uint32)
    start = np.zeros(grid.ncells, np.uint32)
    perm = np.zeros(n, np.int64)
    _load().orc_bin(grid.c(), n, _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(key),
                    _ptr(count), _ptr(start), _ptr(perm))
    return key, count, start, perm


def fluid_flags(grid: Grid, count) -> np.ndarray:
    count = np.ascontiguousarray(count, dtype=np.uint32)
    fluid = np.zeros(grid.ncells, np.uint8)
    _load().orc_fluid_flags(grid.c(), _ptr(count), _ptr(fluid))
    return fluid


def p2g(grid: Grid, pos, vel, return_weights: bool = False):
    """Particle-to-grid (paper Eq. (4)); returns [u, v, w] flat face arrays."""
    pos, vel = _f64(pos), _f64(vel)
    n = pos.shape[1]
    out, wts = [], []
    for a in range(3):
        f = np.zeros(grid.nfaces(a), np.float64)
        w = np.zeros(grid.nfaces(a), np.float64)
        _load().orc_p2g(grid.c(), a, n, _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(vel[a]),
                        _ptr(f), _ptr(w))
        out.append(f)
        wts.append(w)
    return (out, wts) if return_weights else out


def forces_walls(grid: Grid, faces, gravity, dt: float):
    res = []
    for a in range(3):
        f = _f64(faces[a]).copy()
        _load().orc_forces_walls(grid.c(), a, float(gravity[a]), float(dt), _ptr(f))
        res.append(f)
    return res


def divergence(grid: Grid, faces) -> np.ndarray:
    u, v, w = (_f64(f) for f in faces)
    div = np.zeros(grid.ncells, np.float64)
    _load().orc_divergence(grid.c(), _ptr(u), _ptr(v), _ptr(w), _ptr(div))
    return div


def rhs(grid: Grid, fluid, faces, density: float, dt: float) -> np.ndarray:
    fluid = np.ascontiguousarray(fluid, dtype=np.uint8)
    u, v, w = (_f64(f) for f in faces)
    b = np.zeros(grid.ncells, np.float64)
    _load().orc_rhs(grid.c(), _ptr(fluid), _ptr(u), _ptr(v), _ptr(w), float(density), float(dt), _ptr(b))
    return b


def apply_A(grid: Grid, fluid, x) -> np.ndarray:
    fluid = np.ascontiguousarray(fluid, dtype=np.uint8)
    x = _f64(x)
    y = np.zeros(grid.ncells, np.float64)
    _load().orc_apply_A(grid.c(), _ptr(fluid), _ptr(x), _ptr(y))
    return y


@dataclass
class SolveResult:
    p: np.ndarray
    status: int
    iterations: int
    max_r: float
    max_b: float


def pcg(grid: Grid, fluid, b, tol: float, max_iters: int, precond: int = PRECOND_MIC0) -> SolveResult:
    fluid = np.ascontiguousarray(fluid, dtype=np.uint8)
    b = _f64(b)
    p = np.zeros(grid.ncells, np.float64)
    it = ctypes.c_int(0)
    mr = ctypes.c_double(0)
    mb = ctypes.c_double(0)
    st = _load().orc_pcg(grid.c(), _ptr(fluid), _ptr(b), _ptr(p), float(tol), int(max_iters), int(precond),
                         ctypes.byref(it), ctypes.byref(mr), ctypes.byref(mb))
    return SolveResult(p, st, it.value, mr.value, mb.value)


def project(grid: Grid, fluid, p, density: float, dt: float, star):
    fluid = np.ascontiguousarray(fluid, dtype=np.uint8)
    p = _f64(p)
    out = []
    for a in range(3):
        s = _f64(star[a])
        o = np.zeros_like(s)
        _load().orc_project(grid.c(), a, _ptr(fluid), _ptr(p), float(density), float(dt), _ptr(s), _ptr(o))
        out.append(o)
    return out


def interp(grid: Grid, a: int, f, x: float, y: float, z: float) -> float:
    f = _f64(f)
    return _load().orc_interp(grid.c(), a, _ptr(f), float(x), float(y), float(z))


def g2p_advect(grid: Grid, pos, vel, unew, uold, flip_ratio: float, dt: float, flags: int = 0):
    """Grid-to-particle, PIC/FLIP blend, forward Euler and clamp; returns new (pos, vel)."""
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    n = pos.shape[1]
    un = [_f64(f) for f in unew]
    uo = [_f64(f) for f in uold]
    arr_n = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in un])
    arr_o = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in uo])
    _load().orc_g2p_advect(grid.c(), n, _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]),
                           _ptr(vel[0]), _ptr(vel[1]), _ptr(vel[2]), arr_n, arr_o,
                           float(flip_ratio), float(dt), int(flags))
    return pos, vel


def cfl_dt(vel, dx: float, alpha: float, dt_max: float) -> float:
    """CFL time step (Sec. 3.1.4): min(dt_max, alpha dx / max |u_p|), dt_max when all rest."""
    vel = _f64(vel)
    n = vel.shape[1]
    return float(_load().orc_cfl_dt(n, _ptr(vel[0]), _ptr(vel[1]), _ptr(vel[2]), float(dx), float(alpha),
                                    float(dt_max)))


def reseed(grid: Grid, sub: int, seed_value: int, step_index: int, round_fp32: bool, count, start, vel_sorted):
    """Reseeding (Sec. 3.1.2): the particles added to fluid cells holding fewer
    than sub^3 binned particles, in cell order: (pos 3 x m, vel 3 x m, cell m)."""
    count = np.ascontiguousarray(count, dtype=np.uint32)
    start = np.ascontiguousarray(start, dtype=np.uint32)
    vel = _f64(vel_sorted)
    lib = _load()
    null = ctypes.c_void_p(0)
    args = (grid.c(), int(sub), int(seed_value) & (2**64 - 1), int(step_index), int(bool(round_fp32)),
            _ptr(count), _ptr(start), _ptr(vel[0]), _ptr(vel[1]), _ptr(vel[2]))
    m = lib.orc_reseed(*args, null, null, null, null, null, null, null)
    pos_new = np.zeros((3, m))
    vel_new = np.zeros((3, m))
    cell_new = np.zeros(m, dtype=np.uint32)
    if m:
        lib.orc_reseed(*args, _ptr(pos_new[0]), _ptr(pos_new[1]), _ptr(pos_new[2]), _ptr(vel_new[0]),
                       _ptr(vel_new[1]), _ptr(vel_new[2]), _ptr(cell_new))
    return pos_new, vel_new, cell_new


def surface_field(grid: Grid, pos, radius: float, search: float, refine: int = 1) -> np.ndarray:
    """Improved-blobby signed distance (Sec. 3.3.1) at the corners of the
    sampling grid (spacing dx / refine), shape (nz*refine+1, ny*refine+1, nx*refine+1)."""
    pos = _f64(pos)
    shape = (grid.nz * refine + 1, grid.ny * refine + 1, grid.nx * refine + 1)
    phi = np.zeros(shape)
    _load().orc_surface_field(grid.c(), int(refine), float(radius), float(search), pos.shape[1],
                              _ptr(pos[0]), _ptr(pos[1]), _ptr(pos[2]), _ptr(phi))
    return phi


def surface_mesh(grid: Grid, phi, refine: int = 1):
    """Marching cubes (Sec. 3.3.2) of the corner field phi: (vertices (nv, 3),
    unit vertex normals (nv, 3), triangles (nt, 3) vertex indices)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    lib = _load()
    nv = ctypes.c_int64(0)
    null = ctypes.c_void_p(0)
    nt = lib.orc_surface_mesh(grid.c(), int(refine), _ptr(phi), null, null, null, ctypes.byref(nv))
    verts = np.zeros((nv.value, 3))
    normals = np.zeros((nv.value, 3))
    tris = np.zeros((nt, 3), dtype=np.int64)
    lib.orc_surface_mesh(grid.c(), int(refine), _ptr(phi), _ptr(verts), _ptr(normals), _ptr(tris),
                         ctypes.byref(nv))
    return verts, normals, tris


def mc_case_triangles(inside: int) -> np.ndarray:
    """Local-edge triples of the triangles of one cube configuration."""
    buf = np.zeros(48, dtype=np.int32)
    nt = _load().orc_mc_case_triangles(int(inside), _ptr(buf))
    return buf[:3 * nt].reshape(nt, 3)


@dataclass
class Params:
    grid: Grid
    gravity: tuple = (0.0, -9.81, 0.0)
    dt: float = 1.0 / 240.0
    flip_ratio: float = 0.95
    density: float = 1.0
    tol: float = 1e-12
    max_iters: int = 0  # 0 -> 20 * max(nx, ny, nz)
    precond: int = PRECOND_MIC0
    no_projection: bool = False
    advect_particle_vel: bool = False
    # reseeding (Sec. 3.1.2): sub > 0 turns it on; seed, the number of steps
    # done before this one, and whether positions are FP32 values
    reseed_sub: int = 0
    reseed_seed: int = 0
    reseed_step: int = 0
    reseed_fp32: bool = False

    def iters_cap(self):
        g = self.grid
        return self.max_iters if self.max_iters > 0 else 20 * max(g.nx, g.ny, g.nz)


@dataclass
class StepResult:
    key: np.ndarray
    count: np.ndarray
    start: np.ndarray
    perm: np.ndarray
    fluid: np.ndarray
    pos_sorted: np.ndarray
    vel_sorted: np.ndarray
    ids: np.ndarray
    u_old: list
    u_star: list
    b: np.ndarray
    solve: SolveResult
    u_new: list
    pos: np.ndarray
    vel: np.ndarray
    extra: dict = field(default_factory=dict)


def step(prm: Params, pos, vel, ids=None) -> StepResult:
    """One FLIP timestep in FP64, stages in the order given in the module docstring."""
    g = prm.grid
    pos, vel = _f64(pos), _f64(vel)
    n = pos.shape[1]
    if ids is None:
        ids = np.arange(n, dtype=np.uint32)
    key, count, start, perm = bin_particles(g, pos)
    pos_s = np.ascontiguousarray(pos[:, perm])
    vel_s = np.ascontiguousarray(vel[:, perm])
    ids_s = np.ascontiguousarray(np.asarray(ids)[perm])
    fluid = fluid_flags(g, count)
    n_new = 0
    if prm.reseed_sub > 0:
        # new particles follow the existing ones of their cell; ids continue from n
        pos_r, vel_r, cell_r = reseed(g, prm.reseed_sub, prm.reseed_seed, prm.reseed_step, prm.reseed_fp32,
                                      count, start, vel_s)
        n_new = pos_r.shape[1]
        if n_new:
            order = np.argsort(np.concatenate([key[perm], cell_r]), kind="stable")
            pos_s = np.ascontiguousarray(np.concatenate([pos_s, pos_r], axis=1)[:, order])
            vel_s = np.ascontiguousarray(np.concatenate([vel_s, vel_r], axis=1)[:, order])
            ids_s = np.ascontiguousarray(np.concatenate([ids_s, n + np.arange(n_new, dtype=np.uint32)])[order])
            count = count + np.bincount(cell_r, minlength=g.ncells).astype(np.uint32)
            start = (np.cumsum(count, dtype=np.uint64) - count).astype(np.uint32)
    u_old = p2g(g, pos_s, vel_s)
    u_star = forces_walls(g, u_old, prm.gravity, prm.dt)
    b = rhs(g, fluid, u_star, prm.density, prm.dt)
    if prm.no_projection:
        sol = SolveResult(np.zeros(g.ncells), STATUS_CONVERGED, 0, 0.0, float(np.max(np.abs(b), initial=0)))
        u_new = [f.copy() for f in u_star]
    else:
        sol = pcg(g, fluid, b, prm.tol, prm.iters_cap(), prm.precond)
        u_new = project(g, fluid, sol.p, prm.density, prm.dt, u_star)
    flags = ADVECT_PARTICLE_VEL if prm.advect_particle_vel else 0
    pos_n, vel_n = g2p_advect(g, pos_s, vel_s, u_new, u_old, prm.flip_ratio, prm.dt, flags)
    return StepResult(key, count, start, perm, fluid, pos_s, vel_s, ids_s, u_old, u_star, b, sol,
                      u_new, pos_n, vel_n, {"n_reseeded": n_new})
