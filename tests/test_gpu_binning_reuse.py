"""A plain step bins the positions its grid-to-particle writes (keys,
provisional ranks, counts, tile flags) for the next step, which then skips its
own keys pass. Reusing them must change nothing: the results are bitwise
those of a handle stepped straight through, when the reuse is cut between
steps by the surface field's rebinning of the current positions, or by a
batched step (which does not bin for the next step), for FP32 and FP64,
Jacobi and multigrid preconditioning.
"""
import pytest

from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import log
from tests.test_gpu_batch import _assert_same, _sim, _snapshot

pytestmark = pytest.mark.gpu

CASES = [(flip.FLIP_FP32, 0), (flip.FLIP_FP32, flip.FLIP_FLAG_MULTIGRID), (flip.FLIP_FP64, flip.FLIP_FLAG_MULTIGRID)]
IDS = ["fp32-jacobi", "fp32-multigrid", "fp64-multigrid"]


def _through(sc, precision, cfg_flags, steps):
    sim = _sim(sc, precision, cfg_flags)
    sim.step(steps)
    snap = _snapshot(sim)
    sim.close()
    return snap


@pytest.mark.parametrize("precision,cfg_flags", CASES, ids=IDS)
def test_rebinning_between_steps_changes_nothing(precision, cfg_flags):
    sc = inputs.scene("drop64")
    log(f"[reuse] rebin between steps prec={precision} flags={cfg_flags}")
    want = _through(sc, precision, cfg_flags, 4)
    sim = _sim(sc, precision, cfg_flags)
    sim.step(2)
    sim.surface_field(0.5 * sc.dx, 2.0 * sc.dx)  # bins the current positions again
    sim.step(2)
    got = _snapshot(sim)
    sim.close()
    _assert_same(got, want, "rebinned between steps")


@pytest.mark.parametrize("precision,cfg_flags", CASES, ids=IDS)
def test_batched_step_between_plain_steps_changes_nothing(precision, cfg_flags):
    sc = inputs.scene("drop64")
    mg = bool(cfg_flags & flip.FLIP_FLAG_MULTIGRID)
    log(f"[reuse] batched step between prec={precision} mg={mg}")
    want = _through(sc, precision, cfg_flags, 4)
    sim = _sim(sc, precision, cfg_flags)
    sim.step(1)
    b = flip.SlotBatch(1, precision=precision, multigrid=mg, graphs=False, max_dims=(sc.n,) * 3)
    b.attach(0, sim)
    b.step(1)
    b.detach(0)
    b.close()
    sim.step(2)
    got = _snapshot(sim)
    sim.close()
    _assert_same(got, want, "batched step between plain steps")
