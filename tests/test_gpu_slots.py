"""Persistent slot batches (continuous batching): scenes join and leave one
batch between steps without rebuilding it.

Each scene's result must be bitwise the result of stepping the same scene
alone, whatever joins or leaves around it and whatever the batch's step
parity when it joins (direct launches and recorded graphs, FP32 and FP64,
Jacobi and multigrid). Membership changes upload tables but never record
graphs again. Attaching a handle the batch cannot take is refused.
"""
import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import log
from tests.test_gpu_batch import _alone, _assert_same, _scenes, _sim, _snapshot

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graphs,cfg_flags,precision", [
    (False, 0, flip.FLIP_FP32), (True, 0, flip.FLIP_FP32), (True, flip.FLIP_FLAG_MULTIGRID, flip.FLIP_FP32),
    (True, flip.FLIP_FLAG_MULTIGRID, flip.FLIP_FP64)], ids=["direct", "graphs", "graphs-multigrid", "graphs-mg-fp64"])
def test_slot_batch_scenes_match_alone(graphs, cfg_flags, precision):
    scs = _scenes(5, seed=31)
    mg = bool(cfg_flags & flip.FLIP_FLAG_MULTIGRID)
    log(f"[slots] graphs={graphs} mg={mg} prec={precision}: " + ",".join(sc.name for sc in scs))
    b = flip.SlotBatch(4, precision=precision, multigrid=mg, graphs=graphs)
    sims = [_sim(sc, precision, cfg_flags) for sc in scs]
    # schedule: scene -> (batch step at which it joins, steps it takes)
    plan = {0: (0, 6), 1: (0, 3), 2: (1, 4), 3: (3, 2), 4: (4, 3)}
    slot_of, done = {}, {}
    for t in range(7):
        for k, (start, n) in plan.items():
            if start == t:
                slot_of[k] = b.free_slot()
                b.attach(slot_of[k], sims[k])
        assert slot_of, "the plan keeps the batch busy"
        b.step(1)
        for k in list(slot_of):
            start, n = plan[k]
            if t + 1 - start == n:
                b.detach(slot_of.pop(k))
                done[k] = _snapshot(sims[k])
    info = b.info()
    log(f"[slots] steps {info.steps}, graph launches {info.graph_launches}, captures {info.graph_captures}, "
        f"table uploads {info.table_uploads}")
    assert set(done) == set(plan)
    if graphs:
        assert info.graph_launches > info.steps
    assert info.table_uploads >= 4
    b.close()
    for k, sc in enumerate(scs):
        ref = _alone(sc, plan[k][1], precision, cfg_flags)
        _assert_same(done[k], ref, sc.name)
        sims[k].close()


def test_slot_batch_refuses_what_it_cannot_take():
    log("[slots] refusals")
    sc32 = [sc for sc in _scenes(12, seed=5) if sc.n == 32][0]
    b = flip.SlotBatch(2, precision=flip.FLIP_FP32, multigrid=False, graphs=False, max_dims=(32, 32, 32))
    ok = _sim(sc32)
    bad_prec = _sim(sc32, precision=flip.FLIP_FP64)
    bad_mg = _sim(sc32, cfg_flags=flip.FLIP_FLAG_MULTIGRID)
    big = _sim(inputs.scene("drop64"))
    for s in (bad_prec, bad_mg, big):
        with pytest.raises(flip.FlipError) as e:
            b.attach(0, s)
        assert e.value.status == flip.FLIP_E_INVALID
    b.attach(0, ok)
    with pytest.raises(flip.FlipError):
        b.attach(1, ok)            # the same handle twice
    with pytest.raises(flip.FlipError):
        b.attach(0, big)           # an occupied slot
    with pytest.raises(flip.FlipError):
        b.detach(1)                # an empty slot
    with pytest.raises(flip.FlipError):
        b.attach(2, ok)            # out of range
    assert b.step(1) == flip.FLIP_OK
    b.detach(0)
    assert b.step(1) == flip.FLIP_OK   # an empty batch steps nothing
    assert b.info().occupied == 0
    b.close()
    for s in (ok, bad_prec, bad_mg, big):
        s.close()


@pytest.mark.parametrize("mg", [False, True], ids=["jacobi", "multigrid"])
def test_slot_changes_replay_the_recorded_graphs(mg):
    """A scene leaving and another of the same grid taking its slot changes no
    launch's size much: the tables are uploaded again, nothing is recorded
    again, and the scenes' results are bitwise their results alone."""
    cfg_flags = flip.FLIP_FLAG_MULTIGRID if mg else 0
    same = [sc for sc in _scenes(16, seed=8) if sc.n == 48][:3]
    assert len(same) == 3
    log(f"[slots] swap mg={mg}: " + ",".join(sc.name for sc in same))
    b = flip.SlotBatch(2, multigrid=mg, graphs=True)
    sims = [_sim(sc, cfg_flags=cfg_flags) for sc in same]
    b.attach(0, sims[0])
    b.attach(1, sims[1])
    b.step(4)
    # recorded from the batch's second step on: before and after the solve
    # for each particle-buffer parity, the solver chunk (and the short chunk
    # of multigrid batches)
    before = b.info()
    assert before.graph_captures == (6 if mg else 5)
    b.detach(1)
    done1 = _snapshot(sims[1])
    b.attach(1, sims[2])
    b.step(3)
    after = b.info()
    log(f"[slots] captures {before.graph_captures} -> {after.graph_captures}, uploads {before.table_uploads} -> "
        f"{after.table_uploads}, graph launches {after.graph_launches}")
    assert after.graph_captures == before.graph_captures
    assert after.table_uploads == before.table_uploads + 1
    done0, done2 = _snapshot(sims[0]), _snapshot(sims[2])
    b.close()
    _assert_same(done0, _alone(same[0], 7, None, cfg_flags), same[0].name)
    _assert_same(done1, _alone(same[1], 4, None, cfg_flags), same[1].name)
    _assert_same(done2, _alone(same[2], 3, None, cfg_flags), same[2].name)
    for sim in sims:
        sim.close()
