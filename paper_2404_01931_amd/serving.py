"""Continuous-batching server for many independent FLIP scenes on one GPU.

Requests are scenes that arrive over time, each asking for a number of steps.
A request is admitted, in arrival order, when a slot is free and its device
workspace (flip_workspace_bytes) fits in what is left of the HBM budget; a
request larger than the whole budget is rejected. Admitted scenes are
initialised by a preparation thread on a stream of its own, so host-side
seeding and upload overlap the steps of the scenes already on the GPU, and
join the running batch at the next step boundary. The batch is one
persistent slot batch (flip_batch_create_slots), made once: a scene joins by
taking a free slot (flip_batch_attach) and leaves by freeing it
(flip_batch_detach), so membership changes rebuild nothing and the batch's
recorded graphs are replayed throughout. Every step advances all resident
scenes together with one batched step (flip_batch_step: one launch per kernel
for all scenes); scenes that have taken their steps leave at the step
boundary and return their memory to the budget.

Reported: per scene-step latency (the wall time of the batched step it took
part in) p50 / p99, end-to-end scene latency (arrival to last step), queueing
delay, aggregate particle-steps/s over the run, peak resident bytes and
scenes, slot changes, and the batch's graph replays and table uploads.

The GPU work is done by a backend: FlipBackend drives libflipmi through its C
ABI; tests of the scheduling logic use a backend of their own.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float        # seconds after the start of the run
    scene: object         # backend-specific scene description
    steps: int


@dataclass
class _Resident:
    req: Request
    state: object         # backend handle
    nbytes: int
    n_particles: int
    admitted: float
    joined: float = 0.0
    done_steps: int = 0


@dataclass
class ServeReport:
    n_requests: int
    n_completed: int
    n_rejected: int
    wall_s: float
    particle_steps: int
    step_latency_ms: list = field(default_factory=list)   # one entry per batched step
    step_scenes: list = field(default_factory=list)       # resident scenes of each batched step
    scene_latency_s: list = field(default_factory=list)   # arrival -> completion, per scene
    queue_delay_s: list = field(default_factory=list)     # arrival -> admission, per scene
    peak_bytes: int = 0
    peak_scenes: int = 0
    batch_rebuilds: int = 0     # batches made (one persistent slot batch per run)
    slot_changes: int = 0       # scenes attached to or detached from the batch
    status_errors: int = 0
    batch_info: dict = field(default_factory=dict)

    def summary(self) -> dict:
        # every scene-step of a batched step waits for the whole step: weight by scenes
        lat = np.repeat(np.asarray(self.step_latency_ms, np.float64),
                        np.asarray(self.step_scenes, np.int64)) if self.step_latency_ms else np.zeros(0)
        pct = (lambda a, q: float(np.percentile(a, q)) if a.size else None)
        e2e = np.asarray(self.scene_latency_s, np.float64)
        qd = np.asarray(self.queue_delay_s, np.float64)
        return {
            "requests": self.n_requests, "completed": self.n_completed, "rejected": self.n_rejected,
            "wall_s": self.wall_s, "particle_steps": self.particle_steps,
            "particle_steps_per_s": self.particle_steps / self.wall_s if self.wall_s > 0 else None,
            "scene_steps": int(lat.size),
            "step_latency_ms_p50": pct(lat, 50), "step_latency_ms_p99": pct(lat, 99),
            "scene_latency_s_p50": pct(e2e, 50), "scene_latency_s_p99": pct(e2e, 99),
            "queue_delay_s_p50": pct(qd, 50), "queue_delay_s_p99": pct(qd, 99),
            "batched_steps": len(self.step_latency_ms),
            "mean_resident_scenes": float(np.mean(self.step_scenes)) if self.step_scenes else 0.0,
            "peak_resident_scenes": self.peak_scenes, "peak_resident_bytes": self.peak_bytes,
            "batch_rebuilds": self.batch_rebuilds, "slot_changes": self.slot_changes,
            "status_errors": self.status_errors, **self.batch_info,
        }


class Server:
    """FIFO admission by slots and HBM budget; one batched step per tick."""

    def __init__(self, backend, budget_bytes: int, max_slots: int = 64, prep_threads: int = 1,
                 clock=time.perf_counter):
        assert max_slots >= 1 and budget_bytes > 0
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.prep_threads = int(prep_threads)
        self.clock = clock

    def run(self, requests: list[Request]) -> ServeReport:
        be = self.backend
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = deque(reqs)               # not yet arrived
        queue: deque[Request] = deque()     # arrived, waiting for admission
        preparing: list[tuple[Request, int, float, Future]] = []
        resident: list[_Resident] = []
        used = 0
        rep = ServeReport(n_requests=len(reqs), n_completed=0, n_rejected=0, wall_s=0.0, particle_steps=0)
        batch = None
        slot_of: dict[int, int] = {}        # resident scene (rid) -> its slot in the batch
        free_slots = list(range(self.max_slots - 1, -1, -1))
        pool = ThreadPoolExecutor(max_workers=self.prep_threads, initializer=be.prep_thread_init)
        t0 = self.clock()
        try:
            while pending or queue or preparing or resident:
                now = self.clock() - t0
                while pending and pending[0].arrival <= now:
                    queue.append(pending.popleft())
                # admission, in arrival order
                while queue:
                    r = queue[0]
                    need = be.workspace_bytes(r.scene)
                    if need > self.budget:
                        queue.popleft()
                        rep.n_rejected += 1
                        continue
                    if len(resident) + len(preparing) >= self.max_slots or used + need > self.budget:
                        break
                    queue.popleft()
                    used += need
                    rep.queue_delay_s.append(now - r.arrival)
                    preparing.append((r, need, now, pool.submit(be.prepare, r.scene)))
                rep.peak_bytes = max(rep.peak_bytes, used)
                # prepared scenes join at this step boundary
                still = []
                for r, need, adm, fut in preparing:
                    if fut.done():
                        state = fut.result()
                        resident.append(_Resident(r, state, need, be.n_particles(state), adm, self.clock() - t0))
                    else:
                        still.append((r, need, adm, fut))
                preparing = still
                if not resident:
                    if preparing:
                        preparing[0][3].result()   # wait for the first preparation to finish
                    elif pending and not queue:
                        time.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 0.05)))
                    continue
                if batch is None:
                    batch = be.open_batch(self.max_slots)
                    rep.batch_rebuilds += 1
                for s in resident:
                    if s.req.rid not in slot_of:
                        slot_of[s.req.rid] = free_slots.pop()
                        be.attach(batch, slot_of[s.req.rid], s.state)
                        rep.slot_changes += 1
                rep.peak_scenes = max(rep.peak_scenes, len(resident))
                ts = self.clock()
                ok = be.step(batch)
                te = self.clock()
                if not ok:
                    rep.status_errors += 1
                rep.step_latency_ms.append((te - ts) * 1e3)
                rep.step_scenes.append(len(resident))
                left, done = [], []
                for s in resident:
                    s.done_steps += 1
                    rep.particle_steps += s.n_particles
                    (done if s.done_steps >= s.req.steps else left).append(s)
                for s in done:
                    # the scene leaves the batch before its handle goes
                    slot = slot_of.pop(s.req.rid)
                    be.detach(batch, slot)
                    free_slots.append(slot)
                    rep.slot_changes += 1
                    rep.n_completed += 1
                    rep.scene_latency_s.append(te - t0 - s.req.arrival)
                    be.finish(s.state)
                    used -= s.nbytes
                resident = left
        finally:
            if batch is not None:
                rep.batch_info = be.batch_info(batch)
                be.close_batch(batch)
            pool.shutdown(wait=True)
        rep.wall_s = self.clock() - t0
        return rep


class FlipBackend:
    """Scenes of paper_2404_01931_amd.inputs run by libflipmi on the current GPU."""

    def __init__(self, graphs: bool = True, precision=None, keep_results: bool = False, multigrid: bool = False,
                 max_dims=(96, 96, 96)):
        import torch

        from . import flip

        self.flip = flip
        self.torch = torch
        self.graphs = graphs
        self.precision = precision
        self.keep_results = keep_results
        self.multigrid = multigrid
        self.max_dims = tuple(max_dims)   # the largest scene grid the batch takes
        self.cfg_flags = flip.FLIP_FLAG_MULTIGRID if multigrid else 0
        self.results = {}   # scene name -> (pos, vel, ids) at completion, when keep_results
        self.stream = torch.cuda.Stream()   # default priority
        self._local = threading.local()
        self._bytes_cache = {}

    def _cfg(self, scene):
        return self.flip.scene_config(scene, precision=self.precision, flags=self.cfg_flags)

    def workspace_bytes(self, scene) -> int:
        k = scene.name
        if k not in self._bytes_cache:
            cfg, keep = self._cfg(scene)
            self._bytes_cache[k] = self.flip.flip_workspace_bytes(cfg) + 256
        return self._bytes_cache[k]

    def prep_thread_init(self):
        self._local.stream = self.torch.cuda.Stream()

    def prepare(self, scene):
        st = getattr(self._local, "stream", None)
        if st is None:
            self.prep_thread_init()
            st = self._local.stream
        cfg, keep = self._cfg(scene)
        with self.torch.cuda.stream(st):
            sim = self.flip.Simulation(cfg, keep, stream=st)
        sim.stream = self.stream     # stepped on the serving stream from now on
        sim.scene_name = scene.name
        return sim

    def n_particles(self, sim) -> int:
        return sim.n

    def open_batch(self, nslots: int):
        f = self.flip
        prec = f.FLIP_FP64 if self.precision == f.FLIP_FP64 else f.FLIP_FP32
        return f.SlotBatch(nslots, precision=prec, multigrid=self.multigrid, graphs=self.graphs,
                           max_dims=self.max_dims, stream=self.stream)

    def attach(self, batch, slot: int, sim):
        batch.attach(slot, sim)

    def detach(self, batch, slot: int):
        batch.detach(slot)

    def batch_info(self, batch) -> dict:
        i = batch.info()
        return {"batch_steps": i.steps, "graph_launches": i.graph_launches, "graph_captures": i.graph_captures,
                "table_uploads": i.table_uploads}

    def step(self, batch) -> bool:
        st = batch.step(1, allow=(self.flip.FLIP_E_NOT_CONVERGED,))
        batch.stream.synchronize()
        return st == self.flip.FLIP_OK

    def close_batch(self, batch):
        batch.close()

    def finish(self, sim):
        if self.keep_results:
            f = self.flip
            self.results[sim.scene_name] = (sim.read(f.FLIP_FIELD_POS), sim.read(f.FLIP_FIELD_VEL),
                                            sim.read(f.FLIP_FIELD_ID))
        sim.close()
        sim.ws = None


def requests_from_scenes(arrivals_and_scenes) -> list[Request]:
    return [Request(rid=i, arrival=float(t), scene=sc, steps=int(sc.steps))
            for i, (t, sc) in enumerate(arrivals_and_scenes)]
