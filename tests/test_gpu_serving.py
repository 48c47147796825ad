"""The continuous-batching server on the GPU: a short stream of uneven scenes
under an HBM budget that holds only some of them at a time. Every scene must
complete, and its final state must be bitwise the state of the same scene
stepped alone (scenes join and leave batches while others run)."""
import dataclasses

import numpy as np
import pytest

from paper_2404_01931_amd import flip, inputs
from paper_2404_01931_amd.serving import FlipBackend, Server, requests_from_scenes
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graphs,multigrid", [(False, False), (True, False), (True, True)],
                         ids=["direct", "graphs", "graphs-multigrid"])
def test_served_scenes_match_alone(graphs, multigrid):
    stream = inputs.serving_scenes(count=6, seed=21)
    # short requests of uneven length, arriving 5 ms apart
    stream = [(0.005 * i, dataclasses.replace(sc, steps=3 + (i % 3))) for i, (_, sc) in enumerate(stream)]
    reqs = requests_from_scenes(stream)
    be = FlipBackend(graphs=graphs, keep_results=True, multigrid=multigrid)
    sizes = sorted(be.workspace_bytes(r.scene) for r in reqs)
    budget = sizes[-1] + sizes[-2]          # at most two of the largest at once
    log(f"[serving] graphs={graphs} budget={budget} scenes=" + ",".join(r.scene.name for r in reqs))
    rep = Server(be, budget_bytes=budget, max_slots=3).run(reqs)
    s = rep.summary()
    log(f"[serving] {s}")
    assert rep.n_completed == len(reqs) and rep.n_rejected == 0 and rep.status_errors == 0
    assert rep.peak_bytes <= budget and rep.peak_scenes <= 3
    for r in reqs:
        cfg, keep = flip.scene_config(r.scene, flags=flip.FLIP_FLAG_MULTIGRID if multigrid else 0)
        sim = flip.Simulation(cfg, keep)
        sim.step(r.steps)
        ref = (sim.read(flip.FLIP_FIELD_POS), sim.read(flip.FLIP_FIELD_VEL), sim.read(flip.FLIP_FIELD_ID))
        sim.close()
        got = be.results[r.scene.name]
        for a, b in zip(got, ref):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), r.scene.name
