"""Scheduling logic of the continuous-batching server, on the CPU with a
backend that records what the server asks of it (no GPU work)."""
import threading
import time

import pytest

from paper_2404_01931_amd import inputs
from paper_2404_01931_amd.serving import Request, Server, requests_from_scenes


class RecordingBackend:
    def __init__(self, step_s=0.0):
        self.step_s = step_s
        self.lock = threading.Lock()
        self.batches = []          # list of member-name tuples, one per batched step
        self.resident_bytes = []   # bytes held by prepared, unfinished scenes at each step
        self.live = {}
        self.steps_of = {}
        self.admit_order = []
        self.opened = 0
        self.slots = None          # slot -> scene name of the open batch

    def workspace_bytes(self, scene):
        return scene["bytes"]

    def prep_thread_init(self):
        pass

    def prepare(self, scene):
        with self.lock:
            self.live[scene["name"]] = scene["bytes"]
            self.admit_order.append(scene["name"])
        return {"name": scene["name"], "n": scene["n"]}

    def n_particles(self, st):
        return st["n"]

    def open_batch(self, nslots):
        assert self.slots is None, "one persistent batch per run"
        self.opened += 1
        self.slots = [None] * nslots
        return self.slots

    def attach(self, batch, slot, st):
        assert batch is self.slots and batch[slot] is None and st["name"] not in batch
        batch[slot] = st["name"]

    def detach(self, batch, slot):
        assert batch is self.slots and batch[slot] is not None
        batch[slot] = None

    def batch_info(self, batch):
        return {}

    def step(self, batch):
        if self.step_s:
            time.sleep(self.step_s)
        names = tuple(sorted(n for n in batch if n is not None))
        with self.lock:
            self.batches.append(names)
            self.resident_bytes.append(sum(self.live.values()))
        for name in names:
            self.steps_of[name] = self.steps_of.get(name, 0) + 1
        return True

    def close_batch(self, batch):
        assert batch is self.slots
        self.slots = None

    def finish(self, st):
        # a batch refers to its scenes' handles: a scene leaves it first
        assert self.slots is None or st["name"] not in self.slots
        with self.lock:
            del self.live[st["name"]]


def _reqs(specs):
    return [Request(rid=i, arrival=t, scene={"name": f"s{i}", "bytes": b, "n": n}, steps=k)
            for i, (t, b, n, k) in enumerate(specs)]


def test_every_request_completes_with_its_steps():
    specs = [(0.0, 10, 100, 3), (0.0, 20, 200, 5), (0.001, 10, 50, 1), (0.002, 30, 10, 4)]
    be = RecordingBackend()
    rep = Server(be, budget_bytes=1000, max_slots=8).run(_reqs(specs))
    assert rep.n_completed == 4 and rep.n_rejected == 0
    assert be.steps_of == {"s0": 3, "s1": 5, "s2": 1, "s3": 4}
    assert rep.particle_steps == 100 * 3 + 200 * 5 + 50 * 1 + 10 * 4
    s = rep.summary()
    assert s["scene_steps"] == 13 and s["step_latency_ms_p99"] >= s["step_latency_ms_p50"] >= 0.0
    assert len(rep.scene_latency_s) == 4 and len(rep.queue_delay_s) == 4
    assert be.slots is None and be.opened == 1 and rep.batch_rebuilds == 1
    assert rep.slot_changes == 8   # every scene attached once and detached once


def test_budget_and_slots_are_never_exceeded():
    specs = [(0.0, 40, 10, 2 + (i % 3)) for i in range(12)]
    be = RecordingBackend()
    rep = Server(be, budget_bytes=100, max_slots=3).run(_reqs(specs))
    assert rep.n_completed == 12
    assert max(be.resident_bytes) <= 100 and rep.peak_bytes <= 100
    assert max(len(b) for b in be.batches) <= 2          # 40-byte scenes: at most 2 fit in 100 bytes
    rep2 = Server(RecordingBackend(), budget_bytes=10_000, max_slots=3).run(_reqs(specs))
    assert rep2.peak_scenes <= 3


def test_oversize_request_is_rejected_not_fatal():
    specs = [(0.0, 500, 10, 2), (0.0, 10, 10, 2)]
    be = RecordingBackend()
    rep = Server(be, budget_bytes=100, max_slots=4).run(_reqs(specs))
    assert rep.n_rejected == 1 and rep.n_completed == 1 and be.steps_of == {"s1": 2}


def test_admission_follows_arrival_order():
    # a big request at the head blocks smaller later ones until it fits (no overtaking)
    specs = [(0.0, 60, 10, 4), (0.0, 60, 10, 1), (0.0, 10, 10, 1)]
    be = RecordingBackend()
    Server(be, budget_bytes=100, max_slots=4).run(_reqs(specs))
    assert be.admit_order == ["s0", "s1", "s2"]
    first_with_s1 = next(i for i, b in enumerate(be.batches) if "s1" in b)
    assert all("s0" not in b for b in be.batches[first_with_s1:])   # s1 waited for s0's memory


def test_late_arrivals_join_running_batches():
    specs = [(0.0, 10, 10, 40), (0.02, 10, 10, 2)]
    be = RecordingBackend(step_s=0.002)   # s0 runs for about 80 ms
    rep = Server(be, budget_bytes=100, max_slots=4).run(_reqs(specs))
    assert rep.n_completed == 2
    joint = [b for b in be.batches if set(b) == {"s0", "s1"}]
    assert len(joint) == 2           # s1 stepped inside s0's batch, then left
    assert rep.batch_rebuilds == 1   # the one batch throughout: s1 took a slot and gave it back
    assert rep.slot_changes == 4


def test_serving_workload_recipe():
    reqs = requests_from_scenes(inputs.serving_scenes(count=64, seed=5))
    assert len(reqs) == 64
    assert {r.scene.n for r in reqs} <= {32, 48, 64, 96}
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and arr[0] == 0.0
    # Poisson arrivals at 200 / s: mean gap near 5 ms
    gaps = [b - a for a, b in zip(arr, arr[1:])]
    assert 0.002 < sum(gaps) / len(gaps) < 0.01
    assert all(r.steps == 100 for r in reqs)


def test_server_rejects_bad_limits():
    with pytest.raises(AssertionError):
        Server(RecordingBackend(), budget_bytes=0)
    with pytest.raises(AssertionError):
        Server(RecordingBackend(), budget_bytes=10, max_slots=0)
