"""GPU: particle reseeding (FLIP_FLAG_RESEED, paper Sec. 3.1.2), through the C
ABI, against the oracle.

After binning, every fluid cell holding k < sub^3 particles gets sub^3 - k new
ones. Integer results are compared bit for bit: the number of new particles,
their ids, the refilled cell counts and starts. Where the step moves nothing
(no gravity, no projection, particles at rest away from the walls) the new
particles' positions are compared bit for bit too; in full steps everything is
held to the usual step bar against the oracle's step with reseeding.
"""
import dataclasses

import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import by_id, l2_rel, log, params_of, state

pytestmark = pytest.mark.gpu

RS = flip.FLIP_FLAG_RESEED


def _uneven_blob(shape, dx, seed, counts=(1, 2, 3, 5, 7, 8, 9), margin=3):
    """Particles in the interior cells (margin cells from every wall), a random
    number of them per cell, in a shuffled order."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    pos = []
    for k in range(margin, nz - margin):
        for j in range(margin, ny - margin):
            for i in range(margin, nx - margin):
                for _ in range(int(rng.choice(counts))):
                    u = rng.uniform(0.05, 0.95, 3)
                    pos.append(((i + u[0]) * dx, (j + u[1]) * dx, (k + u[2]) * dx))
    pos = np.array(pos).T
    return np.ascontiguousarray(pos[:, rng.permutation(pos.shape[1])])


@pytest.mark.parametrize("prec,shape,dx", [(flip.FLIP_FP64, (16, 12, 10), 1 / 16),
                                           (flip.FLIP_FP32, (20, 12, 17), 1 / 20)])
def test_reseed_still_scene_is_bit_exact(orc, prec, shape, dx):
    log(f"[reseed] still scene precision {prec} shape {shape}")
    pos = _uneven_blob(shape, dx, 3)
    if prec == flip.FLIP_FP32:
        pos = pos.astype(np.float32).astype(np.float64)
    n = pos.shape[1]
    vel = np.zeros_like(pos)
    cfg, keep = flip.make_config(shape, dx, 1 / 240, precision=prec, pos0=pos, vel0=vel, subcells=2, seed=77,
                                 flags=RS | flip.FLIP_FLAG_NO_GRAVITY | flip.FLIP_FLAG_NO_PROJECTION,
                                 capacity=8 * n)
    sim = flip.Simulation(cfg, keep)
    prm = params_of(sim)
    pos0, vel0, ids0 = state(sim)
    sim.step(1)
    st = sim.stats()
    res = orc.step(prm, pos0, vel0, ids0)
    m = res.extra["n_reseeded"]
    log(f"[reseed] {n} particles, {m} new")
    assert m > 0 and st.n_reseeded == m and st.n_particles == n + m
    pos1, vel1, ids1 = state(sim)
    # ids, order, counts and starts: bit for bit
    assert np.array_equal(ids1, res.ids)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), res.count)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_START), res.start)
    # nothing moves: every position, the new ones included, bit for bit
    assert np.array_equal(pos1, res.pos)
    assert np.all(vel1 == 0)
    sim.close()


@pytest.mark.parametrize("prec", [flip.FLIP_FP64, flip.FLIP_FP32])
def test_reseed_transfer_step_velocities(orc, prec):
    """Random velocities, no gravity or projection: the new particles' velocity
    (the cell mean) enters the transfer; the step matches the oracle's."""
    log(f"[reseed] transfer step precision {prec}")
    shape, dx = (16, 16, 16), 1 / 16
    pos = _uneven_blob(shape, dx, 5)
    vel = np.random.default_rng(6).normal(size=pos.shape) * 0.3
    if prec == flip.FLIP_FP32:
        pos = pos.astype(np.float32).astype(np.float64)
        vel = vel.astype(np.float32).astype(np.float64)
    n = pos.shape[1]
    cfg, keep = flip.make_config(shape, dx, 1 / 240, precision=prec, pos0=pos, vel0=vel, subcells=2, seed=5,
                                 flags=RS | flip.FLIP_FLAG_NO_GRAVITY | flip.FLIP_FLAG_NO_PROJECTION,
                                 capacity=8 * n)
    sim = flip.Simulation(cfg, keep)
    prm = params_of(sim)
    pos0, vel0, ids0 = state(sim)
    sim.step(1)
    res = orc.step(prm, pos0, vel0, ids0)
    pos1, vel1, ids1 = state(sim)
    assert np.array_equal(ids1, res.ids)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), res.count)
    ev, ep = l2_rel(vel1, res.vel), l2_rel(pos1, res.pos)
    log(f"[reseed] velocity l2 {ev:.3e} position l2 {ep:.3e}")
    bar = 1e-12 if prec == flip.FLIP_FP64 else 1e-5
    assert ev <= bar and ep <= bar
    sim.close()


@pytest.mark.parametrize("prec,flags", [(flip.FLIP_FP64, 0), (flip.FLIP_FP32, flip.FLIP_FLAG_MULTIGRID),
                                        (flip.FLIP_MIXED, 0)])
def test_reseed_shadowed_splash_steps(orc, prec, flags):
    """A sphere dropping into a pool: each step the oracle, restarted from the
    GPU's state, reseeds and steps; ids and counts exact, velocities to 1e-4."""
    log(f"[reseed] shadowed drop32 precision {prec} flags {flags}")
    sc = dataclasses.replace(inputs.scene("drop64"), n=32, name="drop32")
    # fluid fills well under half the cells, seeded with 8 particles each, and
    # a step adds at most 7 per fluid cell: 16 slots per cell cover 4 steps
    cfg, keep = flip.scene_config(sc, precision=prec, flags=RS | flags, capacity=16 * sc.n**3)
    sim = flip.Simulation(cfg, keep)
    worst, added = 0.0, 0
    for k in range(4):
        prm = params_of(sim)
        pos0, vel0, ids0 = state(sim)
        sim.step(1)
        st = sim.stats()
        assert st.pcg_status == 0
        res = orc.step(prm, pos0, vel0, ids0)
        pos1, vel1, ids1 = state(sim)
        assert st.n_reseeded == res.extra["n_reseeded"]
        added += st.n_reseeded
        assert np.array_equal(ids1, res.ids), k
        assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), res.count)
        e = l2_rel(by_id(vel1, ids1), by_id(res.vel, res.ids))
        worst = max(worst, e)
        assert e <= 1e-4, (k, e)
    log(f"[reseed] drop32: {added} particles added over 4 steps, worst velocity l2 {worst:.3e}")
    assert added > 0
    sim.close()


def test_reseed_capacity_and_refusals(orc):
    log("[reseed] capacity and refusals")
    shape, dx = (12, 12, 12), 1 / 12
    pos = _uneven_blob(shape, dx, 9)
    n = pos.shape[1]
    vel = np.zeros_like(pos)
    # no room for new particles: the step fails before moving anything (with
    # kernel timing on, its timed launches are still collected)
    cfg, keep = flip.make_config(shape, dx, 1 / 240, pos0=pos, vel0=vel, flags=RS | flip.FLIP_FLAG_KERNEL_TIMING)
    sim = flip.Simulation(cfg, keep)
    before = state(sim)
    with pytest.raises(flip.FlipError) as e:
        sim.step(1)
    assert e.value.status == flip.FLIP_E_WORKSPACE
    st = sim.stats()
    assert st.steps == 0 and st.n_reseeded == 0
    assert st.kernel_launches[flip.KERNEL_NAMES.index("bin_keys")] == 1
    after = state(sim)
    assert sim.n == n
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    sim.close()
    # a density the seeding rule cannot take
    cfg, keep = flip.make_config(shape, dx, 1 / 240, pos0=pos, vel0=vel, flags=RS, subcells=0, capacity=9 * n)
    with pytest.raises(flip.FlipError) as e:
        flip.Simulation(cfg, keep)
    assert e.value.status == flip.FLIP_E_INVALID
    # reseeding handles are not batched
    cfg, keep = flip.make_config(shape, dx, 1 / 240, pos0=pos, vel0=vel, flags=RS, capacity=9 * n)
    a = flip.Simulation(cfg, keep)
    with pytest.raises(flip.FlipError) as e:
        flip.Batch([a])
    assert e.value.status == flip.FLIP_E_INVALID
    a.close()
