"""GPU: flip_surface_mesh_noalloc (marching cubes with the library's own
device scratch, for callers that cannot allocate) against flip_surface_mesh
(the same kernels with a caller workspace), through the C ABI.

Two calls in a row on the same GPU, the second on a smaller sampling grid
(the scratch keeps the first call's contents). Vertex and triangle arrays
must be identical (same kernels on the same field); vertex normals are summed
with atomics, so their last bits depend on the order of the adds: they must
agree within the rounding of those sums: per vertex with m triangles,
2 m sqrt(3) u (sum of the weighted unit normals' magnitudes) / |their sum|
+ 8 u (u the unit roundoff; the two orders each round m - 1 adds per
component, then normalise).
A sampling grid beyond the scratch's limit is refused before anything runs.
"""
import ctypes
import dataclasses

import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _normal_bound(v, t, unit):
    """Per vertex: 2 m sqrt(3) u sum|n_i / A_i| / |sum n_i / A_i| + 8 u over its m triangles (FP64, host)."""
    A, B, C = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(B - A, C - A)
    area2 = np.linalg.norm(cr, axis=1)
    ok = area2 > 0
    w = np.zeros_like(cr)
    w[ok] = cr[ok] / area2[ok, None] / (0.5 * area2[ok, None])  # unit normal over the area
    mag = np.zeros(len(v))
    vec = np.zeros((len(v), 3))
    m = np.zeros(len(v))
    for k in range(3):
        np.add.at(mag, t[:, k], np.linalg.norm(w, axis=1))
        np.add.at(vec, t[:, k], w)
        np.add.at(m, t[:, k], 1.0)
    norm = np.linalg.norm(vec, axis=1)
    return 2 * m * np.sqrt(3.0) * unit * mag / np.maximum(norm, 1e-300) + 8 * unit


def _compare(sim, phi, refine, out=None):
    verts, normals, tris = sim.surface_mesh_device(phi, refine)
    v2, n2, t2 = sim.surface_mesh_noalloc_device(phi, refine, out=out)
    sim.stream.synchronize()
    v, n, t = verts.cpu().numpy(), normals.cpu().numpy(), tris.cpu().numpy()
    v2, n2, t2 = v2.cpu().numpy(), n2.cpu().numpy(), t2.cpu().numpy()
    log(f"[noalloc] refine {refine}: {len(v)} vertices, {len(t)} triangles (no-alloc {len(v2)}, {len(t2)})")
    assert len(t) > 0
    assert np.array_equal(t, t2)
    assert np.array_equal(v, v2)
    unit = 2.0**-53 if v.dtype == np.float64 else 2.0**-24
    bound = _normal_bound(v.astype(np.float64), t, unit)
    err = np.linalg.norm(n.astype(np.float64) - n2.astype(np.float64), axis=1)
    log(f"[noalloc] normals: max err {err.max():.2e}, worst err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("prec", [flip.FLIP_FP32, flip.FLIP_FP64])
def test_noalloc_mesh_matches_workspace_mesh_twice(prec):
    log(f"[noalloc] dam32 precision {prec}")
    cfg, keep = flip.scene_config(inputs.scene("dam32"), precision=prec, flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    sim.step(3)
    dx = cfg.dx
    # first call: 65^3 sampling grid; outputs counted and allocated by the binding
    phi2 = sim.surface_field_device(0.5 * dx, 2 * dx, 2)
    _compare(sim, phi2, 2)
    # second call, smaller input: 33^3 sampling grid, into preallocated outputs
    # larger than the mesh (the call writes only the mesh's entries)
    phi1 = sim.surface_field_device(0.5 * dx, 2 * dx, 1)
    dt = phi1.dtype
    big = 200000
    out = (sim.torch.full((big, 3), -7.0, dtype=dt, device="cuda"),
           sim.torch.full((big, 3), -7.0, dtype=dt, device="cuda"),
           sim.torch.full((big, 3), -1, dtype=sim.torch.int32, device="cuda"))
    _compare(sim, phi1, 1, out=out)
    sim.close()


def test_noalloc_mesh_refuses_grids_beyond_its_scratch():
    """129^3 corners need more than FLIP_MESH_SCRATCH_MAX_BYTES of scratch:
    FLIP_E_WORKSPACE, counts untouched, nothing enqueued."""
    log("[noalloc] limit")
    shape, dx = (128, 128, 128), 1 / 128
    pos, vel = inputs.random_particles(shape, 64, seed=2, lo=(0.4,) * 3, hi=(0.6,) * 3, dx=dx)
    cfg, keep = flip.make_config(shape, dx, 1 / 240, pos0=pos, vel0=vel)
    sim = flip.Simulation(cfg, keep)
    lib = flip.load()
    wb = ctypes.c_size_t(0)
    assert lib.flip_surface_mesh_workspace_bytes(sim.h, 1, ctypes.byref(wb)) == flip.FLIP_OK
    assert wb.value > flip.FLIP_MESH_SCRATCH_MAX_BYTES
    phi = sim.torch.zeros(16, dtype=sim.torch.float32, device="cuda")  # never read: refused first
    nv, nt = ctypes.c_int64(-5), ctypes.c_int64(-5)
    null = ctypes.c_void_p(0)
    rc = lib.flip_surface_mesh_noalloc(sim.h, ctypes.c_void_p(phi.data_ptr()), 1, null, null, 0, null, 0,
                                       ctypes.byref(nv), ctypes.byref(nt), ctypes.c_void_p(sim.stream.cuda_stream))
    assert rc == flip.FLIP_E_WORKSPACE
    assert nv.value == -5 and nt.value == -5
    # argument errors come first, as in flip_surface_mesh
    assert lib.flip_surface_mesh_noalloc(sim.h, null, 1, null, null, 0, null, 0, ctypes.byref(nv),
                                         ctypes.byref(nt), null) == flip.FLIP_E_INVALID
    sim.close()
