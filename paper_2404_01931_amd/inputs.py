"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle's tests.

This module holds scene descriptions and random-number draws only; it contains
none of the method's arithmetic. The scenes stand in for the paper's benchmark
scenes (dam break and water drop, Sec. 4, Table 1), which the paper describes
only by particle count and grid size:

* ``dam32``      dam break, 32^3, fluid block x < 0.5, y < 0.5 (all z), FP64
* ``dam128``     dam break, 128^3, fluid block x < 0.4, y < 0.6 (all z), FP32
* ``drop256``    drop into a pool, 256^3: pool y < 0.3 plus a sphere of radius
                 0.15 at (0.5, 0.7, 0.5) moving at (0, -1, 0), FP32
* ``drop256_mixed`` the same scene with the mixed-precision solver
* ``drop64``     the drop scene downscaled to 64^3 (mixed-precision comparison size)
* ``drop128``    the drop scene at 128^3 (bounded sample for the CPU baseline)

Every scene uses 2 x 2 x 2 jittered subcells per fluid cell (paper Fig. 3),
gravity (0, -9.81, 0) and solid walls on all six domain faces.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

INF = float("inf")


@dataclass(frozen=True)
class RegionSpec:
    kind: str  # "box" | "sphere"
    lo: tuple = (-INF, -INF, -INF)
    hi: tuple = (INF, INF, INF)
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    vel: tuple = (0.0, 0.0, 0.0)


@dataclass(frozen=True)
class Scene:
    name: str
    n: int                      # cells per axis (cubic domain [0, n*dx]^3)
    regions: tuple
    seed: int
    precision: str              # "fp32" | "fp64" | "mixed"
    dt: float
    flip_ratio: float
    tol: float
    steps: int
    sub: int = 2
    gravity: tuple = (0.0, -9.81, 0.0)
    density: float = 1.0
    ir_tol: float = 1e-8
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def dx(self) -> float:
        return 1.0 / self.n


def dam(n: int, x_hi: float, y_hi: float, **kw) -> Scene:
    reg = (RegionSpec("box", hi=(x_hi, y_hi, INF)),)
    return Scene(regions=reg, n=n, **kw)


def double_dam(n: int, width: float, height: float, **kw) -> Scene:
    """Two water columns against opposite walls (the paper's double dam break,
    Table 1; its geometry is not given: columns x < width and x >= 1 - width,
    y < height, all z)."""
    reg = (RegionSpec("box", hi=(width, height, INF)), RegionSpec("box", lo=(1.0 - width, -INF, -INF),
                                                                  hi=(INF, height, INF)))
    return Scene(regions=reg, n=n, **kw)


def drop(n: int, **kw) -> Scene:
    reg = (RegionSpec("box", hi=(INF, 0.3, INF)),
           RegionSpec("sphere", center=(0.5, 0.7, 0.5), radius=0.15, vel=(0.0, -1.0, 0.0)))
    return Scene(regions=reg, n=n, **kw)


SCENES = {
    "dam32": dam(32, 0.5, 0.5, name="dam32", seed=1, precision="fp64", dt=1 / 240,
                 flip_ratio=0.95, tol=1e-6, steps=20),
    "dam128": dam(128, 0.4, 0.6, name="dam128", seed=2, precision="fp32", dt=1 / 480,
                  flip_ratio=0.95, tol=1e-6, steps=50),
    "drop256": drop(256, name="drop256", seed=3, precision="fp32", dt=1 / 960,
                    flip_ratio=0.97, tol=1e-6, steps=30),
    # mixed precision: tol is the tolerance of each FP32 inner solve (relative to the
    # residual it starts from); the FP64 refinement stops at ir_tol. With 3e-5 two
    # refinements reach 1e-8 (with 1e-4 the second one lands just short of it, so
    # a third runs)
    "drop256_mixed": drop(256, name="drop256_mixed", seed=4, precision="mixed", dt=1 / 960,
                          flip_ratio=0.97, tol=3e-5, steps=30, ir_tol=1e-8),
    "drop64": drop(64, name="drop64", seed=4, precision="fp32", dt=1 / 960,
                   flip_ratio=0.97, tol=1e-6, steps=30),
    "drop128": drop(128, name="drop128", seed=3, precision="fp32", dt=1 / 960,
                    flip_ratio=0.97, tol=1e-6, steps=30),
    "ddam32": double_dam(32, 0.25, 0.5, name="ddam32", seed=6, precision="fp64", dt=1 / 240,
                         flip_ratio=0.95, tol=1e-6, steps=20),
    "ddam128": double_dam(128, 0.25, 0.5, name="ddam128", seed=6, precision="fp32", dt=1 / 480,
                          flip_ratio=0.95, tol=1e-6, steps=50),
}


def describe(sc: Scene) -> str:
    """Short description of a scene's layout."""
    kinds = [r.kind for r in sc.regions]
    if "sphere" in kinds:
        return "drop into pool"
    return "double dam break" if len(kinds) == 2 else "dam break"


def scene(name: str, **overrides) -> Scene:
    s = SCENES[name]
    return replace(s, **overrides) if overrides else s


def serving_scenes(count: int = 512, seed: int = 5):
    """Serving workload: independent dam/drop scenes, side drawn from {32, 48, 64, 96},
    100 steps at dt = 1/240, layout seed 1000 + scene id, Poisson arrivals at 200/s."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([32, 48, 64, 96], size=count)
    kinds = rng.integers(0, 2, size=count)
    gaps = rng.exponential(1.0 / 200.0, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for s in range(count):
        n = int(sides[s])
        if kinds[s] == 0:
            sc = dam(n, 0.5, 0.5, name=f"serve{s}_dam{n}", seed=1000 + s, precision="fp32",
                     dt=1 / 240, flip_ratio=0.95, tol=1e-6, steps=100)
        else:
            sc = drop(n, name=f"serve{s}_drop{n}", seed=1000 + s, precision="fp32",
                      dt=1 / 240, flip_ratio=0.97, tol=1e-6, steps=100)
        out.append((float(arrivals[s]), sc))
    return out


def random_particles(shape, count: int, seed: int, lo=None, hi=None, vel_scale: float = 1.0,
                     dx: float | None = None):
    """Uniformly random positions in the box [lo, hi) (world units) and normal velocities.

    ``shape`` is (nx, ny, nz); by default the box is the whole domain shrunk by
    one cell on every side. Returns (pos (3, n), vel (3, n)) as float64.
    """
    nx, ny, nz = shape
    if dx is None:
        dx = 1.0 / max(shape)
    L = np.array([nx, ny, nz], np.float64) * dx
    lo = np.full(3, dx) if lo is None else np.asarray(lo, np.float64)
    hi = L - dx if hi is None else np.asarray(hi, np.float64)
    rng = np.random.default_rng(seed)
    pos = lo[:, None] + (hi - lo)[:, None] * rng.random((3, count))
    vel = vel_scale * rng.standard_normal((3, count))
    return pos, vel
