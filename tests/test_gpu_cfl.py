"""GPU: the CFL time step (FLIP_FLAG_ADAPTIVE_DT, paper Sec. 3.1.4), through the
C ABI, against the oracle.

Each step takes dt = min(config dt, cfl * dx / |u|max) from the particles'
speeds at its start. The step's dt (reported in the stats) must equal the
oracle's CFL rule evaluated on the same particle velocities bit for bit (both
evaluate the speeds in FP64 in the same order), and the step with it must
match the oracle's step with that dt to the usual bar.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import l2_rel, log, params_of, state

pytestmark = pytest.mark.gpu

CFL = flip.FLIP_FLAG_ADAPTIVE_DT


def _drop32(prec, cfl):
    sc = dataclasses.replace(inputs.scene("drop64"), n=32, name="drop32")
    # a small CFL number so that the rule, not the cap, sets dt (the sphere falls at 1)
    return flip.scene_config(sc, precision=prec, flags=CFL, cfl=cfl)


@pytest.mark.parametrize("prec,bar", [(flip.FLIP_FP64, 1e-4), (flip.FLIP_FP32, 1e-4)])
def test_cfl_steps_against_oracle(orc, prec, bar):
    log(f"[cfl] precision {prec}")
    cfg, keep = _drop32(prec, 0.01)
    sim = flip.Simulation(cfg, keep)
    prm = params_of(sim)
    worst, dts = 0.0, []
    for k in range(4):
        pos0, vel0, ids0 = state(sim)
        dt_ref = orc.cfl_dt(vel0, cfg.dx, cfg.cfl, cfg.dt)
        sim.step(1)
        st = sim.stats()
        assert st.dt == dt_ref, (k, st.dt, dt_ref)
        assert st.dt < cfg.dt  # the rule, not the cap
        dts.append(st.dt)
        pos1, vel1, ids1 = state(sim)
        res = orc.step(dataclasses.replace(prm, dt=dt_ref), pos0, vel0, ids0)
        assert np.array_equal(res.ids, ids1)
        e = l2_rel(vel1, res.vel)
        worst = max(worst, e)
        assert e <= bar, (k, e)
    log(f"[cfl] dts {dts}, worst velocity l2 error {worst:.3e}")
    # the particles accelerate under gravity: the step shrinks
    assert dts[-1] < dts[0]
    sim.close()


def test_cfl_cap_and_fixed_dt():
    log("[cfl] cap and fixed dt")
    # a large CFL number: the configured dt caps the step
    cfg, keep = _drop32(flip.FLIP_FP32, 3.0)
    sim = flip.Simulation(cfg, keep)
    sim.step(1)
    assert sim.stats().dt == cfg.dt
    sim.close()
    # without the flag every step takes the configured dt
    cfg, keep = flip.scene_config(inputs.scene("dam32"))
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    assert sim.stats().dt == cfg.dt
    sim.close()


def test_cfl_refusals():
    log("[cfl] refusals")
    cfg, keep = _drop32(flip.FLIP_FP32, 0.0)
    with pytest.raises(flip.FlipError) as e:
        flip.Simulation(cfg, keep)
    assert e.value.status == flip.FLIP_E_INVALID
    cfg, keep = _drop32(flip.FLIP_FP32, 3.0)
    a = flip.Simulation(cfg, keep)
    with pytest.raises(flip.FlipError) as e:
        flip.Batch([a])
    assert e.value.status == flip.FLIP_E_INVALID
    a.close()
