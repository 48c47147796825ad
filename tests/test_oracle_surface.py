"""Pins of the oracle's surface scalar field (paper Sec. 3.3.1, improved blobbies).

The field is checked against what its definition fixes in cases worked out by
hand: the exact signed distance of one isolated particle's sphere, a two-particle
value computed from the kernel by hand, the midpoint of a symmetric pair, the
kernel's support, the reading for corners far from every particle, and exact
relations between sampling grids (refinement, translation).
"""
import numpy as np

import oracle as O


def _one(x):
    return np.array(x, dtype=np.float64).reshape(3, 1)


def _corners(g, refine=1):
    h = g.dx / refine
    K, J, I = np.meshgrid(np.arange(g.nz * refine + 1), np.arange(g.ny * refine + 1),
                          np.arange(g.nx * refine + 1), indexing="ij")
    return I * h, J * h, K * h


def test_isolated_particle_gives_the_exact_sphere_distance():
    g = O.Grid(8, 8, 8, 0.125)
    r, R = 0.05, 0.25
    p = (0.53, 0.41, 0.47)
    phi = O.surface_field(g, _one(p), r, R)
    X, Y, Z = _corners(g)
    d = np.sqrt((X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2)
    near = d < R
    assert near.sum() > 8
    assert np.allclose(phi[near], d[near] - r, rtol=0, atol=1e-15)
    assert np.all(phi[~near] == R)  # reading: no particle in reach -> outside, phi = R


def test_two_particle_value_worked_by_hand():
    # corner at (0.5, 0.5, 0.5); particle A on the corner (s = 0, k = 1), B at
    # distance R/2 along x (s = 1/2, k = (3/4)^3 = 27/64): the weighted centre is
    # R/2 * (27/64) / (91/64) = 27 R / 182 from the corner, so phi = 27 R / 182 - r
    g = O.Grid(4, 4, 4, 0.25)
    r, R = 0.1, 0.25
    pos = np.array([[0.5, 0.5 + R / 2], [0.5, 0.5], [0.5, 0.5]])
    phi = O.surface_field(g, pos, r, R)
    assert abs(phi[2, 2, 2] - (27 * R / 182 - r)) < 1e-15


def test_symmetric_pair_centres_on_the_corner_and_support_is_strict():
    g = O.Grid(4, 4, 4, 0.25)
    r, R = 0.1, 0.25
    a = 0.0625
    pos = np.array([[0.5 - a, 0.5 + a], [0.5, 0.5], [0.5, 0.5]])
    phi = O.surface_field(g, pos, r, R)
    assert phi[2, 2, 2] == -r
    # a particle at exactly R weighs nothing; just inside R it alone sets phi
    phi = O.surface_field(g, _one((0.5 + R, 0.5, 0.5)), r, R)
    assert phi[2, 2, 2] == R
    d = R * (1 - 2.0**-20)
    phi = O.surface_field(g, _one((0.5 + d, 0.5, 0.5)), r, R)
    assert abs(phi[2, 2, 2] - (d - r)) < 1e-15


def test_refinement_and_translation_are_exact():
    g = O.Grid(6, 5, 4, 0.125)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0.1, 0.5, size=(3, 200))
    pos = np.round(pos * 2**20) / 2**20  # dyadic, so shifts are exact
    r, R = 0.06, 0.25
    phi1 = O.surface_field(g, pos, r, R, refine=1)
    phi2 = O.surface_field(g, pos, r, R, refine=2)
    assert np.array_equal(phi2[::2, ::2, ::2], phi1)  # same corners, same values
    # shifting every particle by one sampling step shifts the field by one node
    h = g.dx
    phis = O.surface_field(g, pos + np.array([[h], [0.0], [0.0]]), r, R)
    assert np.allclose(phis[:, :, 1:], phi1[:, :, :-1], rtol=0, atol=1e-14)


def test_ball_of_particles_has_its_zero_level_near_the_ball_surface():
    # a jittered lattice (spacing dx/2) filling a ball of radius 0.3; particle
    # radius = the spacing: inside negative, outside positive, and along the
    # axes the zero crossing lies within one cell of the ball's surface
    n, dx = 32, 1 / 32
    g = O.Grid(n, n, n, dx)
    rng = np.random.default_rng(1)
    s = dx / 2
    ax = np.arange(s / 2, 1, s)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    pts = pts + rng.uniform(-s / 4, s / 4, pts.shape)
    c, rb = 0.5, 0.3
    pts = pts[:, np.sum((pts - c) ** 2, axis=0) < rb * rb]
    phi = O.surface_field(g, pts, s, 2 * dx)
    assert phi[16, 16, 16] < 0 and phi[0, 0, 0] > 0
    line = phi[16, 16, :]  # along x through the centre
    xs = np.arange(n + 1) * dx
    i = np.nonzero((line[:-1] > 0) & (line[1:] <= 0))[0][0]
    x0 = xs[i] + dx * line[i] / (line[i] - line[i + 1])
    assert abs((c - x0) - rb) < dx
