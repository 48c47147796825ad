"""GPU: the surface scalar field (flip_surface_field, paper Sec. 3.3.1), through
the C ABI, against the oracle.

Every corner of small sampling grids is compared with the oracle's field, which
evaluates the definition against every particle; at a 128^3 scene, corners
sampled near the surface and at random are compared with the oracle evaluated
on the particles around each of them. Tolerances: 1e-12 R in FP64; 1e-5 R in
FP32 (sums of a few hundred weighted offsets in single precision).
"""
import ctypes
import dataclasses

import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import grid_of, log

pytestmark = pytest.mark.gpu


def _scene(prec, n=16):
    sc = dataclasses.replace(inputs.scene("dam32"), n=n, name=f"dam{n}")
    return flip.scene_config(sc, precision=prec, flags=flip.FLIP_FLAG_MULTIGRID)


@pytest.mark.parametrize("prec,refine", [(flip.FLIP_FP64, 1), (flip.FLIP_FP64, 2), (flip.FLIP_FP32, 1),
                                         (flip.FLIP_FP32, 2)])
def test_surface_field_every_corner_against_oracle(orc, prec, refine):
    log(f"[surface] precision {prec} refine {refine}")
    cfg, keep = _scene(prec)
    sim = flip.Simulation(cfg, keep)
    sim.step(3)  # a moving, uneven surface
    dx = cfg.dx
    r, R = 0.5 * dx, 2.0 * dx
    phi = sim.surface_field(r, R, refine).astype(np.float64)
    pos = sim.read(flip.FLIP_FIELD_POS).astype(np.float64)
    ref = orc.surface_field(grid_of(sim), pos, r, R, refine)
    assert phi.shape == ref.shape
    err = np.abs(phi - ref).max()
    inside, outside = (ref < 0).sum(), (ref == R).sum()
    log(f"[surface] {phi.size} corners ({inside} inside, {outside} beyond reach), max error {err / R:.2e} R")
    assert inside > 0 and outside > 0
    assert err <= (1e-12 if prec == flip.FLIP_FP64 else 1e-5) * R
    # the call bins the particles: the id field stays a permutation
    ids = sim.read(flip.FLIP_FIELD_ID)
    assert np.array_equal(np.sort(ids), np.arange(sim.n))
    sim.close()


def test_surface_field_sampled_corners_at_128(orc):
    log("[surface] drop128 sampled corners")
    cfg, keep = flip.scene_config(inputs.scene("drop128"), flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    dx = cfg.dx
    r, R = 0.5 * dx, 2.0 * dx
    phi = sim.surface_field(r, R, 1).astype(np.float64)
    pos = sim.read(flip.FLIP_FIELD_POS).astype(np.float64)
    rng = np.random.default_rng(0)
    near = np.argwhere(np.abs(phi) < dx)
    pick = np.concatenate([near[rng.choice(len(near), 48, replace=False)],
                           rng.integers(0, phi.shape[0], size=(16, 3))])
    worst = 0.0
    for K, J, I in pick:
        x = np.array([I, J, K]) * dx
        # the particles within reach, moved so the corner is node (3, 3, 3) of a
        # 6^3 grid (a shift by whole cells)
        sel = np.all(np.abs(pos - x[:, None]) < R + dx, axis=0)
        shift = (np.array([I, J, K]) - 3) * dx
        local = pos[:, sel] - shift[:, None]
        ref = orc.surface_field(flip_grid(6, dx), np.ascontiguousarray(local), r, R)[3, 3, 3]
        worst = max(worst, abs(phi[K, J, I] - ref))
    log(f"[surface] 64 sampled corners, max error {worst / R:.2e} R")
    assert worst <= 1e-5 * R
    sim.close()


def flip_grid(n, dx):
    import oracle as O

    return O.Grid(n, n, n, dx)


def test_surface_field_argument_errors():
    log("[surface] argument errors")
    cfg, keep = _scene(flip.FLIP_FP32, 8)
    sim = flip.Simulation(cfg, keep)
    lib = flip.load()
    nbytes = ctypes.c_size_t(0)
    assert lib.flip_surface_field_bytes(sim.h, 0, ctypes.byref(nbytes)) == flip.FLIP_E_INVALID
    assert lib.flip_surface_field_bytes(sim.h, 1, ctypes.byref(nbytes)) == flip.FLIP_OK
    assert nbytes.value == 9**3 * 4
    buf = sim.torch.empty(nbytes.value, dtype=sim.torch.uint8, device="cuda")
    ptr, st = ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(sim.stream.cuda_stream)
    assert lib.flip_surface_field(sim.h, 0.0, 0.2, 1, ptr, nbytes.value, st) == flip.FLIP_E_INVALID
    assert lib.flip_surface_field(sim.h, 0.1, float("nan"), 1, ptr, nbytes.value, st) == flip.FLIP_E_INVALID
    assert lib.flip_surface_field(sim.h, 0.1, 0.2, 17, ptr, nbytes.value, st) == flip.FLIP_E_INVALID
    assert lib.flip_surface_field(sim.h, 0.1, 0.2, 1, ptr, nbytes.value - 1, st) == flip.FLIP_E_INVALID
    assert lib.flip_surface_field(sim.h, 0.1, 0.2, 1, ptr, nbytes.value, st) == flip.FLIP_OK
    sim.stream.synchronize()
    sim.close()
