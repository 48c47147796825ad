"""Helpers for the GPU parity tests: run the library through its C ABI and feed
the oracle the same inputs (the GPU's own state, converted exactly to float64)."""
import sys

import numpy as np

import oracle as O
from paper_2404_01931_amd import flip


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grid_of(sim):
    nx, ny, nz = sim.shape
    return O.Grid(nx, ny, nz, sim.cfg.dx)


def params_of(sim, tol=1e-12, precond=O.PRECOND_MIC0):
    c = sim.cfg
    return O.Params(grid=grid_of(sim), gravity=tuple(c.gravity) if not (c.flags & flip.FLIP_FLAG_NO_GRAVITY)
                    else (0.0, 0.0, 0.0), dt=c.dt, flip_ratio=c.flip_ratio, density=c.density, tol=tol,
                    max_iters=100000, precond=precond,
                    no_projection=bool(c.flags & flip.FLIP_FLAG_NO_PROJECTION),
                    advect_particle_vel=bool(c.flags & flip.FLIP_FLAG_ADVECT_PARTICLE_VEL),
                    reseed_sub=c.subcells_per_axis if c.flags & flip.FLIP_FLAG_RESEED else 0,
                    reseed_seed=c.seed, reseed_step=int(sim.stats().steps),
                    reseed_fp32=c.precision != flip.FLIP_FP64)


def state(sim):
    """(pos, vel, ids) of the handle as float64 / uint32 numpy arrays."""
    return (sim.read(flip.FLIP_FIELD_POS).astype(np.float64), sim.read(flip.FLIP_FIELD_VEL).astype(np.float64),
            sim.read(flip.FLIP_FIELD_ID))


def max_rel(a, b, floor=1e-30):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def l2_rel(a, b, floor=1e-30):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0:
        return 0.0
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))


def by_id(arr, ids):
    """Reorder columns of arr (3, n) so that column i holds particle id i."""
    out = np.empty_like(arr)
    out[:, ids] = arr
    return out
