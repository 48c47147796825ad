"""Batched stepping (the serving form): several scenes of uneven grid sizes
advanced by one launch per kernel.

Each scene's result in a batch must be bitwise the result of stepping the
same scene alone: the batched kernels run the plain kernels' code with the
same per-scene work split and the same fixed-order reductions. Checked with
direct launches and with recorded HIP graphs (replayed from the second step
on, over both particle-buffer phases), for FP32 and FP64, for a scene that
moves from one batch to another (continuous batching), and against the FP64
oracle for one step of a batched scene.
"""
import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import l2_rel, log, params_of, state

pytestmark = pytest.mark.gpu


def _scenes(count=5, seed=11):
    return [sc for _, sc in inputs.serving_scenes(count=count, seed=seed)]


def _sim(sc, precision=None, cfg_flags=0):
    cfg, keep = flip.scene_config(sc, precision=precision, flags=cfg_flags)
    return flip.Simulation(cfg, keep)


def _snapshot(sim):
    return {
        "pos": sim.read(flip.FLIP_FIELD_POS), "vel": sim.read(flip.FLIP_FIELD_VEL),
        "id": sim.read(flip.FLIP_FIELD_ID), "p": sim.read(flip.FLIP_FIELD_PRESSURE),
        "u": sim.read(flip.FLIP_FIELD_U_NEW), "iters": sim.stats().pcg_iterations,
        "steps": sim.stats().steps, "status": sim.stats().pcg_status,
    }


def _alone(sc, steps, precision=None, cfg_flags=0):
    sim = _sim(sc, precision, cfg_flags)
    sim.step(steps)
    snap = _snapshot(sim)
    sim.close()
    return snap


def _assert_same(a, b, what):
    for k in ["pos", "vel", "id", "p", "u"]:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, (what, k)
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (what, k)
    for k in ["iters", "steps", "status"]:
        assert a[k] == b[k], (what, k, a[k], b[k])


@pytest.mark.parametrize("flags,cfg_flags", [(0, 0), (flip.FLIP_BATCH_GRAPHS, 0),
                                              (0, flip.FLIP_FLAG_MULTIGRID),
                                              (flip.FLIP_BATCH_GRAPHS, flip.FLIP_FLAG_MULTIGRID)],
                         ids=["direct", "graphs", "direct-multigrid", "graphs-multigrid"])
def test_batch_matches_alone_bitwise(flags, cfg_flags):
    scs = _scenes(5)
    steps = 5
    log(f"[batch] alone vs mix flags={flags} cfg_flags={cfg_flags}: " + ", ".join(s.name for s in scs))
    ref = [_alone(sc, steps, cfg_flags=cfg_flags) for sc in scs]
    sims = [_sim(sc, cfg_flags=cfg_flags) for sc in scs]
    batch = flip.Batch(sims, flags=flags)
    for _ in range(steps):
        assert batch.step(1) == flip.FLIP_OK
    for sc, sim, r in zip(scs, sims, ref):
        _assert_same(_snapshot(sim), r, sc.name)
    batch.close()
    for s in sims:
        s.close()


def test_batch_fp64_matches_alone_bitwise():
    scs = _scenes(3, seed=12)
    log("[batch] fp64: " + ", ".join(s.name for s in scs))
    ref = [_alone(sc, 3, flip.FLIP_FP64) for sc in scs]
    sims = [_sim(sc, flip.FLIP_FP64) for sc in scs]
    batch = flip.Batch(sims, flags=flip.FLIP_BATCH_GRAPHS)
    assert batch.step(3) == flip.FLIP_OK
    for sc, sim, r in zip(scs, sims, ref):
        _assert_same(_snapshot(sim), r, sc.name)
    batch.close()
    for s in sims:
        s.close()


def test_scene_moving_between_batches_matches_alone():
    """Continuous batching: scene B steps 3 times with A, then 4 times with C
    (which joins late and leaves early) and 2 more with nobody."""
    a, b, c = _scenes(3, seed=13)
    log(f"[batch] membership change: {a.name} {b.name} {c.name}")
    ref_b = _alone(b, 9)
    ref_c = _alone(c, 4)
    sa, sb, sc_ = _sim(a), _sim(b), _sim(c)
    b1 = flip.Batch([sa, sb], flags=flip.FLIP_BATCH_GRAPHS)
    b1.step(3)
    b1.close()
    b2 = flip.Batch([sc_, sb])
    b2.step(4)
    b2.close()
    b3 = flip.Batch([sb], flags=flip.FLIP_BATCH_GRAPHS)
    b3.step(2)
    b3.close()
    _assert_same(_snapshot(sb), ref_b, b.name)
    _assert_same(_snapshot(sc_), ref_c, c.name)
    for s in (sa, sb, sc_):
        s.close()


def test_stepping_outside_the_batch_is_refused():
    a, b = _scenes(2, seed=14)
    sa, sb = _sim(a), _sim(b)
    batch = flip.Batch([sa, sb])
    batch.step(1)
    sa.step(1)  # the batch's tables now point at the wrong particle buffers
    with pytest.raises(flip.FlipError) as e:
        batch.step(1)
    assert e.value.status == flip.FLIP_E_STATE
    batch.close()
    for s in (sa, sb):
        s.close()


def test_batched_step_against_oracle(orc):
    scs = [s for s in _scenes(6, seed=15)]
    small = min(scs, key=lambda s: s.n)
    log(f"[batch] oracle check of {small.name} in a batch of {len(scs)}")
    sims = [_sim(sc) for sc in scs]
    k = scs.index(small)
    pos0, vel0, ids0 = state(sims[k])
    batch = flip.Batch(sims, flags=flip.FLIP_BATCH_GRAPHS)
    batch.step(1)
    pos1, vel1, ids1 = state(sims[k])
    res = orc.step(params_of(sims[k]), pos0, vel0, ids0)
    assert np.array_equal(res.ids, ids1)
    assert l2_rel(vel1, res.vel) <= 1e-4
    batch.close()
    for s in sims:
        s.close()
