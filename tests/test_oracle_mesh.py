"""Pins of the oracle's marching cubes (paper Sec. 3.3.2).

Checked against what a correct isosurface mesh must satisfy, independently of
the triangulation rule's code: every one of the 256 cube configurations gives
triangles on crossing edges only, whose free edges are exactly the crossings
joined face by face and whose normals point up the field; a sphere's mesh is
closed and consistently oriented (every directed edge once, Euler
characteristic 2), its area and enclosed volume approach the sphere's, its
vertex normals approach the radial direction; a linear field puts every vertex
exactly on the plane; interpolated vertex positions are worked by hand.
"""
import itertools
import math

import numpy as np

import oracle as O


def _edge_corners(e):
    axis, q = e // 4, e % 4
    c0 = [0, 0, 0]
    others = [d for d in range(3) if d != axis]
    c0[others[0]], c0[others[1]] = q & 1, q >> 1
    c1 = list(c0)
    c1[axis] = 1
    return c0, c1


def _trilinear_grad(vals, x):
    g = np.zeros(3)
    for q in range(8):
        c = [(q >> d) & 1 for d in range(3)]
        for d in range(3):
            term = vals[q]
            for e in range(3):
                if e == d:
                    term *= 1.0 if c[e] else -1.0
                else:
                    term *= x[e] if c[e] else 1 - x[e]
            g[d] += term
    return g


def test_every_cube_configuration_is_consistent():
    for case in range(256):
        inside = [(case >> q) & 1 for q in range(8)]
        crossing = set()
        for e in range(12):
            a, b = _edge_corners(e)
            qa = a[0] + 2 * a[1] + 4 * a[2]
            qb = b[0] + 2 * b[1] + 4 * b[2]
            if inside[qa] != inside[qb]:
                crossing.add(e)
        tris = O.mc_case_triangles(case)
        if case in (0, 255):
            assert len(tris) == 0
            continue
        assert len(tris) > 0
        used = set(tris.ravel().tolist())
        assert used == crossing, case  # every crossing carries a vertex, nothing else does
        # free (boundary) edges of the triangle fan lie on cube faces: both
        # endpoints' edges share a face
        count = {}
        for t in tris:
            for k in range(3):
                u, v = int(t[k]), int(t[(k + 1) % 3])
                key = (min(u, v), max(u, v))
                count[key] = count.get(key, 0) + 1
        for (u, v), n in count.items():
            assert n in (1, 2)
            if n == 1:
                cu, cv = set(map(tuple, _edge_corners(u))), set(map(tuple, _edge_corners(v)))
                pts = np.array(list(cu | cv))
                assert any(np.all(pts[:, d] == pts[0, d]) for d in range(3)), (case, u, v)
        # normals point up the field (corner values -1 inside, +1 outside)
        vals = [-1.0 if inside[q] else 1.0 for q in range(8)]
        mid = {e: np.mean(np.array(_edge_corners(e), dtype=float), axis=0) for e in range(12)}
        for t in tris:
            A, B, C = mid[t[0]], mid[t[1]], mid[t[2]]
            n = np.cross(B - A, C - A)
            assert np.dot(n, _trilinear_grad(vals, (A + B + C) / 3)) > 0, (case, t)


def test_single_inside_corner_vertices_worked_by_hand():
    g = O.Grid(1, 1, 1, 0.5)
    phi = np.ones((2, 2, 2))
    phi[0, 0, 0] = -1.0   # corner (0,0,0) inside
    phi[0, 0, 1] = 3.0    # x neighbour: t = 1/4
    phi[0, 1, 0] = 1.0    # y neighbour: t = 1/2
    phi[1, 0, 0] = 0.25   # z neighbour: t = 4/5
    v, nrm, tri = O.surface_mesh(g, phi)
    assert v.shape == (3, 3) and tri.shape == (1, 3)
    # vertices in edge order: x, y, z edges of corner 0
    assert np.allclose(v, [[0.125, 0, 0], [0, 0.25, 0], [0, 0, 0.4]], atol=1e-15)
    n = np.cross(v[tri[0, 1]] - v[tri[0, 0]], v[tri[0, 2]] - v[tri[0, 0]])
    assert np.all(n > 0)  # away from the inside corner
    assert np.allclose(nrm, n / np.linalg.norm(n))


def test_inverse_area_vertex_normals_worked_by_hand():
    """Sec. 3.3.2 weights each face normal at a vertex by the inverse of the
    face's area. Two inside corners joined along x give one quad of crossing
    vertices, split into two triangles of different areas and normals; at the
    two vertices they share, normalise(n1/A1 + n2/A2) differs from the
    area-weighted and the unweighted sums, so either slip fails here."""
    g = O.Grid(1, 1, 1, 1.0)
    phi = np.ones((2, 2, 2))   # phi[K, J, I]
    phi[0, 0, 0] = -1.0        # corner (0,0,0) inside
    phi[0, 0, 1] = -1.0        # corner (1,0,0) inside
    phi[0, 1, 0] = 1.0         # (0,0,0) -> (0,1,0): t = 1/2
    phi[1, 0, 0] = 3.0         # (0,0,0) -> (0,0,1): t = 1/4
    phi[0, 1, 1] = 0.25        # (1,0,0) -> (1,1,0): t = 4/5
    phi[1, 0, 1] = 1.0         # (1,0,0) -> (1,0,1): t = 1/2
    v, nrm, tri = O.surface_mesh(g, phi)
    # vertices in edge order (y and z edges of corner 0, then of corner 1)
    P = np.array([[0, 0.5, 0], [0, 0, 0.25], [1, 0.8, 0], [1, 0, 0.5]])
    assert np.allclose(v, P, atol=1e-15)
    assert tri.shape == (2, 3)
    assert sorted(set(tri.ravel().tolist())) == [0, 1, 2, 3]
    shared = sorted(set(tri[0].tolist()) & set(tri[1].tolist()))
    assert len(shared) == 2
    # each triangle's cross product: twice its area times its unit normal
    cr = [np.cross(P[t[1]] - P[t[0]], P[t[2]] - P[t[0]]) for t in tri]
    area = [0.5 * np.linalg.norm(c) for c in cr]
    unit = [c / np.linalg.norm(c) for c in cr]
    assert abs(area[0] - area[1]) > 0.05 * max(area)
    assert np.dot(unit[0], unit[1]) < 0.999

    def nz(w):
        return w / np.linalg.norm(w)

    inv = nz(unit[0] / area[0] + unit[1] / area[1])
    for s in shared:
        assert np.allclose(nrm[s], inv, atol=1e-14)
        assert np.linalg.norm(nrm[s] - nz(unit[0] * area[0] + unit[1] * area[1])) > 1e-3
        assert np.linalg.norm(nrm[s] - nz(unit[0] + unit[1])) > 1e-3
    for t in range(2):
        for q in set(tri[t].tolist()) - set(shared):
            assert np.allclose(nrm[q], unit[t], atol=1e-14)
    # out of the fluid: the inside corners sit on the edge y = z = 0
    assert np.all(nrm[:, 1] > 0) and np.all(nrm[:, 2] > 0)


def test_plane_vertices_lie_on_the_plane():
    g = O.Grid(6, 5, 4, 0.25)
    x = np.arange(7) * 0.25
    phi = np.broadcast_to(x - 0.8, (5, 6, 7)).copy()
    v, nrm, tri = O.surface_mesh(g, phi)
    assert np.allclose(v[:, 0], 0.8, atol=1e-15)
    assert np.allclose(nrm, [1.0, 0.0, 0.0], atol=1e-12)
    assert len(tri) == 2 * 5 * 4  # two triangles per cube the plane crosses


def test_sphere_mesh_is_closed_oriented_and_converges():
    c, rho = np.array([0.5, 0.47, 0.52]), 0.3
    areas, vols = [], []
    for n in (16, 32, 64):
        g = O.Grid(n, n, n, 1.0 / n)
        K, J, I = np.meshgrid(*(np.arange(n + 1) / n,) * 3, indexing="ij")
        phi = np.sqrt((I - c[0]) ** 2 + (J - c[1]) ** 2 + (K - c[2]) ** 2) - rho
        v, nrm, tri = O.surface_mesh(g, phi)
        # closed and consistently oriented: each directed edge exactly once, and its reverse too
        directed = {}
        for t in tri:
            for k in range(3):
                e = (int(t[k]), int(t[(k + 1) % 3]))
                directed[e] = directed.get(e, 0) + 1
        assert all(m == 1 for m in directed.values())
        assert all((b, a) in directed for (a, b) in directed)
        E = len(directed) // 2
        assert len(v) - E + len(tri) == 2
        A, B, C = v[tri[:, 0]], v[tri[:, 1]], v[tri[:, 2]]
        cr = np.cross(B - A, C - A)
        areas.append(0.5 * np.linalg.norm(cr, axis=1).sum())
        vols.append(np.einsum("ij,ij->i", A, np.cross(B, C)).sum() / 6)
        radial = (v - c) / np.linalg.norm(v - c, axis=1)[:, None]
        assert np.min(np.einsum("ij,ij->i", nrm, radial)) > (0.95 if n > 16 else 0.9)
    A0, V0 = 4 * math.pi * rho**2, 4 / 3 * math.pi * rho**3
    errs = [abs(a - A0) / A0 for a in areas]
    verrs = [abs(w - V0) / V0 for w in vols]
    assert all(w > 0 for w in vols)  # outward orientation encloses positive volume
    assert errs[-1] < 0.01 and verrs[-1] < 0.005
    assert errs[2] < errs[0] and verrs[2] < verrs[0]
