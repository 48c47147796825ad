"""Pins of the oracle's reseeding (paper Sec. 3.1.2, closing paragraph).

Each check is made against what the reading fixes, computed independently of
the oracle: counts by brute force over the cells, positions by exact rational
arithmetic (cell and subcell of every new particle), velocities against an
exactly rounded sum, and the step as a whole against the invariants a
transfer-only step with uniform velocity must keep.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _particles_with_counts(grid, counts, rng):
    """Particles placed uniformly inside each cell, counts[c] of them in cell c,
    in a shuffled order; velocities random."""
    pos, cells = [], []
    for c, k in enumerate(counts):
        i, j, kk = c % grid.nx, (c // grid.nx) % grid.ny, c // (grid.nx * grid.ny)
        for _ in range(int(k)):
            u = rng.uniform(0.02, 0.98, 3)
            pos.append(((i + u[0]) * grid.dx, (j + u[1]) * grid.dx, (kk + u[2]) * grid.dx))
            cells.append(c)
    pos = np.array(pos, dtype=np.float64).T.reshape(3, -1)
    order = rng.permutation(pos.shape[1])
    vel = rng.normal(size=pos.shape)
    return np.ascontiguousarray(pos[:, order]), vel, np.array(cells)[order]


def _binned(grid, pos, vel):
    key, count, start, perm = O.bin_particles(grid, pos)
    return key, count, start, perm, np.ascontiguousarray(vel[:, perm])


def _cell_ijk(grid, c):
    return c % grid.nx, (c // grid.nx) % grid.ny, c // (grid.nx * grid.ny)


def test_reseed_fills_sparse_fluid_cells_up_to_the_density():
    g = O.Grid(6, 5, 4, 1.0 / 6.0)  # a cell size that is not a power of two
    rng = np.random.default_rng(11)
    counts = rng.choice([0, 0, 1, 2, 3, 5, 7, 8, 9, 12], size=g.ncells)
    pos, vel, _ = _particles_with_counts(g, counts, rng)
    _, count, start, _, vel_s = _binned(g, pos, vel)
    assert np.array_equal(count, counts)
    sub, target = 2, 8
    pn, vn, cn = O.reseed(g, sub, 1234, 3, False, count, start, vel_s)

    # counts: air and full cells untouched, every other fluid cell topped up
    want = {c: target - int(k) for c, k in enumerate(counts) if 0 < k < target}
    assert pn.shape[1] == sum(want.values())
    assert np.all(np.diff(cn.astype(np.int64)) >= 0)  # cell order
    got = np.bincount(cn, minlength=g.ncells)
    for c in range(g.ncells):
        assert got[c] == want.get(c, 0)

    # positions: inside the cell, and the t-th new particle of a cell that
    # held k lies in jitter subcell k + t (x-fastest), by exact arithmetic
    dx = Fraction(g.dx)
    t_of = {}
    for m in range(pn.shape[1]):
        c = int(cn[m])
        t = t_of.get(c, 0)
        t_of[c] = t + 1
        s = int(counts[c]) + t
        sub_idx = (s % sub, (s // sub) % sub, s // (sub * sub))
        for a, ijk in enumerate(_cell_ijk(g, c)):
            q = Fraction(pn[a, m]) / dx
            assert math.floor(q) == ijk
            assert math.floor((q - ijk) * sub) == sub_idx[a]

    # velocities: the mean of the cell's binned particles (exactly rounded sum,
    # so the oracle's running sum may differ by a few ulps)
    for m in range(pn.shape[1]):
        c = int(cn[m])
        k = int(count[c])
        for a in range(3):
            exact = math.fsum(vel_s[a, start[c]:start[c] + k]) / k
            assert vn[a, m] == pytest.approx(exact, rel=1e-14, abs=1e-15)

    # the same call gives the same particles; another step other positions
    pn2, vn2, cn2 = O.reseed(g, sub, 1234, 3, False, count, start, vel_s)
    assert np.array_equal(pn, pn2) and np.array_equal(vn, vn2) and np.array_equal(cn, cn2)
    pn3, _, cn3 = O.reseed(g, sub, 1234, 4, False, count, start, vel_s)
    assert np.array_equal(cn, cn3) and not np.any(pn == pn3)


def test_reseed_single_particle_cell_copies_its_velocity_and_density_one_adds_nothing():
    g = O.Grid(3, 3, 3, 0.25)
    counts = np.zeros(g.ncells, dtype=int)
    counts[13] = 1
    rng = np.random.default_rng(2)
    pos, vel, _ = _particles_with_counts(g, counts, rng)
    _, count, start, _, vel_s = _binned(g, pos, vel)
    pn, vn, cn = O.reseed(g, 3, 7, 0, False, count, start, vel_s)
    assert pn.shape[1] == 26 and np.all(cn == 13)
    assert np.all(vn == vel_s[:, :1])  # the mean of one value is that value
    pn, _, _ = O.reseed(g, 1, 7, 0, False, count, start, vel_s)  # one particle per cell asked
    assert pn.shape[1] == 0
    empty = np.zeros(g.ncells, dtype=np.uint32)
    pn, _, _ = O.reseed(g, 2, 7, 0, False, empty, empty, np.zeros((3, 0)))
    assert pn.shape[1] == 0


def test_reseed_jitter_is_uniform_within_the_subcell():
    g = O.Grid(40, 10, 10, 0.05)
    counts = np.ones(g.ncells, dtype=int)
    rng = np.random.default_rng(5)
    pos, vel, _ = _particles_with_counts(g, counts, rng)
    _, count, start, _, vel_s = _binned(g, pos, vel)
    sub = 4
    pn, _, cn = O.reseed(g, sub, 99, 1, False, count, start, vel_s)
    assert pn.shape[1] == g.ncells * (sub**3 - 1)
    ijk = np.stack(_cell_ijk(g, cn.astype(np.int64)))
    frac = (pn / g.dx - ijk) * sub
    off = frac - np.floor(frac)
    assert off.min() >= 0.0 and off.max() < 1.0
    # 252000 uniform samples per axis: mean 1/2 and variance 1/12 within a few sigma
    for a in range(3):
        assert abs(off[a].mean() - 0.5) < 5 * math.sqrt(1 / 12 / off.shape[1])
        assert abs(off[a].var() - 1 / 12) < 0.003


def _splitmix64(seed, counter):
    """Element `counter` of the SplitMix64 sequence of `seed` (Steele, Lea &
    Flood 2014), vectorised in wrapping uint64 arithmetic."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def test_reseed_fp32_positions_are_float_values_inside_their_cells():
    # a long row of cells with a non-dyadic cell size: FP32 rounding of the
    # jittered points lands some of them on the far side of a cell face, and
    # those must come back into their cell
    g = O.Grid(4000, 2, 2, 0.1)
    counts = np.ones(g.ncells, dtype=int)
    rng = np.random.default_rng(8)
    pos, vel, _ = _particles_with_counts(g, counts, rng)
    pos = pos.astype(np.float32).astype(np.float64)
    vel = vel.astype(np.float32).astype(np.float64)
    _, count, start, _, vel_s = _binned(g, pos, vel)
    sub, seed, step = 4, 2024, 0
    pn, vn, cn = O.reseed(g, sub, seed, step, True, count, start, vel_s)
    m = pn.shape[1]
    assert m == g.ncells * 63
    assert np.array_equal(pn.astype(np.float32).astype(np.float64), pn)
    assert np.array_equal(vn.astype(np.float32).astype(np.float64), vn)
    assert np.array_equal(vn, np.repeat(vel_s, 63, axis=1))
    # every new particle bins into its own cell (exact floor of the binning)
    assert np.array_equal(O.cell_keys(g, pn), cn)

    # the x coordinate before rounding, from the jitter rule written out here
    c = cn.astype(np.int64)
    s = np.tile(np.arange(1, 64), g.ncells)
    i = c % g.nx
    ctr = 3 * (sub**3 * (g.ncells * (step + 1) + c) + s)
    xi = (_splitmix64(seed, ctr) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    x64 = ((s % sub + xi) / sub + i) * g.dx
    x32 = x64.astype(np.float32).astype(np.float64)
    dx = Fraction(g.dx)
    cand = np.nonzero(np.abs(x32 / g.dx - np.round(x32 / g.dx)) < 1e-3)[0]
    out = [q for q in cand if math.floor(Fraction(x32[q]) / dx) != i[q]]
    assert len(out) > 0, "the case must exercise the move back into the cell"
    for q in out:
        assert math.floor(Fraction(pn[0, q]) / dx) == i[q]
        # moved by the fewest representable steps: the value next to it is outside
        nxt = np.nextafter(np.float32(pn[0, q]), np.float32(x32[q]))
        assert math.floor(Fraction(float(nxt)) / dx) != i[q]
    inside = np.setdiff1d(np.arange(m), np.array(out, dtype=np.int64))
    assert np.array_equal(pn[0, inside], x32[inside])


def test_step_with_reseeding_keeps_a_uniform_flow_uniform():
    """A transfer-only step (no gravity, no projection) of a uniform velocity
    field: reseeded particles take that velocity, every particle moves by
    dt * v, ids stay unique and count up from n."""
    g = O.Grid(8, 8, 8, 1.0 / 8.0)
    rng = np.random.default_rng(4)
    counts = np.zeros((8, 8, 8), dtype=int)
    counts[2:6, 2:6, 2:6] = rng.choice([1, 3, 8, 10], size=(4, 4, 4))
    counts = counts.reshape(-1)
    pos, _, _ = _particles_with_counts(g, counts, rng)
    n = pos.shape[1]
    v = np.array([0.25, -0.5, 0.125])
    vel = np.repeat(v[:, None], n, axis=1)
    prm = O.Params(grid=g, gravity=(0.0, 0.0, 0.0), dt=1.0 / 64, no_projection=True, reseed_sub=2,
                   reseed_seed=42, reseed_step=0)
    ids = np.arange(n, dtype=np.uint32)[::-1].copy()
    res = O.step(prm, pos, vel, ids)
    m = res.extra["n_reseeded"]
    assert m == int(sum(8 - k for k in counts if 0 < k < 8))
    assert res.pos.shape[1] == n + m
    assert np.array_equal(np.sort(res.ids), np.arange(n + m))
    assert np.all(res.vel == v[:, None])
    # the new particles, found by id, sit where reseeding put them, moved by dt v
    pn, _, cn = O.reseed(g, 2, 42, 0, False, *O.bin_particles(g, pos)[1:3], np.repeat(v[:, None], n, 1))
    new = np.argsort(res.ids)[n:]
    assert np.allclose(res.pos[:, new], pn + prm.dt * v[:, None], rtol=0, atol=1e-15)
    # post-reseed counts: every fluid cell at or above the density, sorted order kept
    assert np.array_equal(res.count, np.where((counts > 0) & (counts < 8), 8, counts))
    assert np.all(np.diff(O.cell_keys(g, res.pos_sorted).astype(np.int64)) >= 0)
