"""GPU: marching cubes (flip_surface_mesh, paper Sec. 3.3.2), through the C ABI,
against the oracle.

The GPU meshes its own scalar field; the oracle meshes the same field (read
back). Inside/outside decisions are taken on the same values, so the vertex
count, the triangle count and every triangle's vertex indices must be equal.
In FP64 the GPU's mesh is also compared end to end with the oracle's mesh of
the oracle's own field; in FP32 the inside/outside decisions (integers decided
by floating point) are taken on the kernel's FP32 values, so the comparison is
made on the GPU's field.
Vertices are bit-exact in FP64 (same operations) and within 4 FP32 roundings
of the largest coordinate in FP32; vertex normals (summed with atomics) within 1e-9 in FP64; in FP32
within 1e-5 + 8 (max vertex error) / (smallest altitude of a triangle at the
vertex), since the inverse-area weights let the smallest triangle at a vertex
set its normal.
The 128^3 case meshes the whole field at full size.
"""
import ctypes
import dataclasses

import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import grid_of, log

pytestmark = pytest.mark.gpu


def _mesh_and_compare(orc, sim, refine):
    dx = sim.cfg.dx
    phi = sim.surface_field_device(0.5 * dx, 2 * dx, refine)
    verts, normals, tris = sim.surface_mesh_device(phi, refine)
    sim.stream.synchronize()
    phi_h = phi.cpu().numpy().astype(np.float64)
    v_ref, n_ref, t_ref = orc.surface_mesh(grid_of(sim), phi_h, refine)
    v, n, t = verts.cpu().numpy().astype(np.float64), normals.cpu().numpy().astype(np.float64), tris.cpu().numpy()
    fp64 = sim.cfg.precision == flip.FLIP_FP64
    log(f"[mesh] refine {refine}: {len(v)} vertices, {len(t)} triangles (oracle {len(v_ref)}, {len(t_ref)})")
    assert len(t) > 0
    assert v.shape == v_ref.shape and t.shape == t_ref.shape
    assert np.array_equal(t, t_ref)
    h = dx / refine
    ev = np.abs(v - v_ref).max()
    en = np.abs(n - n_ref).max()
    log(f"[mesh] max vertex error {ev / h:.2e} h, max normal error {en:.2e}")
    if fp64:
        assert np.array_equal(v, v_ref)
        assert en <= 1e-9
        # end to end: the oracle's own field from the particle positions, then
        # its mesh (the two fields differ by rounding, far from any sign change)
        pos = sim.read(flip.FLIP_FIELD_POS).astype(np.float64)
        phi_o = orc.surface_field(grid_of(sim), pos, 0.5 * dx, 2 * dx, refine)
        v_o, n_o, t_o = orc.surface_mesh(grid_of(sim), phi_o, refine)
        assert np.array_equal(t, t_o)
        e2v, e2n = np.abs(v - v_o).max() / h, np.abs(n - n_o).max()
        log(f"[mesh] against the oracle's own field: vertices {e2v:.2e} h, normals {e2n:.2e}")
        assert e2v <= 1e-10 and e2n <= 1e-6
    else:
        # (I + t) h in FP32: a few roundings at the coordinate's magnitude
        assert ev <= 4 * 2.0**-24 * (np.abs(v_ref).max() + h)
        # a vertex normal follows its smallest triangle (inverse-area weights),
        # whose unit normal turns by up to about 2 (vertex error) / (its
        # smallest altitude): the bound per vertex is that over the triangles
        # at the vertex, from the oracle's mesh, with a margin of 4
        A, B, C = v_ref[t_ref[:, 0]], v_ref[t_ref[:, 1]], v_ref[t_ref[:, 2]]
        area2 = np.linalg.norm(np.cross(B - A, C - A), axis=1)
        lmax = np.max([np.linalg.norm(B - A, axis=1), np.linalg.norm(C - B, axis=1),
                       np.linalg.norm(A - C, axis=1)], axis=0)
        alt = area2 / lmax
        amin = np.full(len(v_ref), np.inf)
        for k in range(3):
            np.minimum.at(amin, t_ref[:, k], alt)
        bound = 1e-5 + 8 * max(ev, 1e-12) / amin
        err = np.linalg.norm(n - n_ref, axis=1)
        log(f"[mesh] FP32 normals: {np.mean(err <= 1e-4):.5f} of vertices within 1e-4, worst err / bound "
            f"{np.max(err / bound):.3f}")
        assert np.all(err <= bound)
    return v, t


@pytest.mark.parametrize("prec,refine", [(flip.FLIP_FP64, 1), (flip.FLIP_FP64, 2), (flip.FLIP_FP32, 1),
                                         (flip.FLIP_FP32, 2)])
def test_mesh_small_scene_against_oracle(orc, prec, refine):
    log(f"[mesh] dam16 precision {prec} refine {refine}")
    sc = dataclasses.replace(inputs.scene("dam32"), n=16, name="dam16")
    cfg, keep = flip.scene_config(sc, precision=prec, flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    sim.step(3)
    v, t = _mesh_and_compare(orc, sim, refine)
    # orientation is consistent: no directed edge twice
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    assert len(np.unique(e, axis=0)) == len(e)
    sim.close()


def test_mesh_full_field_at_128(orc):
    log("[mesh] drop128 full field")
    cfg, keep = flip.scene_config(inputs.scene("drop128"), flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    _mesh_and_compare(orc, sim, 1)
    sim.close()


def test_mesh_counts_and_capacity():
    log("[mesh] counts and capacity")
    sc = dataclasses.replace(inputs.scene("dam32"), n=8, name="dam8")
    cfg, keep = flip.scene_config(sc)
    sim = flip.Simulation(cfg, keep)
    phi = sim.surface_field_device(0.5 * cfg.dx, 2 * cfg.dx, 1)
    lib = flip.load()
    wb = ctypes.c_size_t(0)
    assert lib.flip_surface_mesh_workspace_bytes(sim.h, 1, ctypes.byref(wb)) == flip.FLIP_OK
    work = sim.torch.empty(wb.value, dtype=sim.torch.uint8, device="cuda")
    st = ctypes.c_void_p(sim.stream.cuda_stream)
    nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    null = ctypes.c_void_p(0)
    pw, pp = ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(phi.data_ptr())
    assert lib.flip_surface_mesh(sim.h, pp, 1, pw, wb.value, null, null, 0, null, 0, ctypes.byref(nv),
                                 ctypes.byref(nt), st) == flip.FLIP_OK
    assert nv.value > 0 and nt.value > 0
    # a workspace one byte short, and outputs too small for the mesh
    assert lib.flip_surface_mesh(sim.h, pp, 1, pw, wb.value - 1, null, null, 0, null, 0, ctypes.byref(nv),
                                 ctypes.byref(nt), st) == flip.FLIP_E_WORKSPACE
    out = sim.torch.empty(3 * nv.value * 4, dtype=sim.torch.uint8, device="cuda")
    tri = sim.torch.empty(3 * nt.value * 4, dtype=sim.torch.uint8, device="cuda")
    po, pt = ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tri.data_ptr())
    assert lib.flip_surface_mesh(sim.h, pp, 1, pw, wb.value, po, po, nv.value, pt, nt.value - 1, ctypes.byref(nv),
                                 ctypes.byref(nt), st) == flip.FLIP_E_WORKSPACE
    # only some outputs given
    assert lib.flip_surface_mesh(sim.h, pp, 1, pw, wb.value, po, null, nv.value, pt, nt.value, ctypes.byref(nv),
                                 ctypes.byref(nt), st) == flip.FLIP_E_INVALID
    assert lib.flip_surface_mesh_workspace_bytes(sim.h, 0, ctypes.byref(wb)) == flip.FLIP_E_INVALID
    sim.stream.synchronize()
    sim.close()
