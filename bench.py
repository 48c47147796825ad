"""Benchmark: FLIP timestep throughput on one MI355X.

Workload: the 256^3 drop-into-pool scene (pool y < 0.3 plus a sphere of radius
0.15 at (0.5, 0.7, 0.5) falling at 1 m/s; 8 jittered particles per fluid cell,
42,266,944 particles; FP32; dt = 1/960; FLIP ratio 0.97; PCG tolerance 1e-6).
Inputs are synthetic and seeded and already resident in HBM when timing starts.

A step is one full pass of the hot path (binning, particle-to-grid, forces and
walls, right-hand side, PCG solve, projection, grid-to-particle and advection).
Prints ONE JSON line with particle-steps/s (timed on a handle without kernel
timing), the roofline figures of the dominant kernel (algorithmic bytes per
launch over its average duration, from HIP events on a second handle of the
same scene), a serving leg (a stream of independent scenes through the
continuous-batching server, beside the plain path on the same scenes), and
the FP64 oracle timed on the host as a CPU baseline (one step of the same
scene, one thread). The headline uses the multigrid-preconditioned CG; the
Jacobi-preconditioned CG on the same scene is measured too and reported
beside it (`jacobi_pcg_same_scene`), with the roofline of its dominant
kernel. `precision_forms` reports the mixed-precision solve (FP32 vectors,
FP64 reductions, refinement to 1e-8) against the FP64 solve to the same
tolerance and the plain FP32 solve, each with its FP64 true residual and the
divergence the projection leaves.

Usage: python bench.py [--gpus 1] [--steps 30] [--warmup 3] [--scene drop256]
                       [--solver multigrid|jacobi] [--no-second-solver]
                       [--serving-scenes 512] [--serving-only] [--no-cpu-baseline]
                       [--no-precision-forms]
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mg_coarse_cells(nx: int, ny: int, nz: int) -> int:
    """Cells of the multigrid's coarse levels (each axis halved, ceil, until
    no axis has more than 8 cells), stored dense."""
    total = 0
    while True:
        nx, ny, nz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
        total += nx * ny * nz
        if max(nx, ny, nz) <= 8:
            return total


def algorithmic_bytes(kind: str, rb: int, n: int, cells: int, faces: list, fluid: float,
                      coarse: int = 0, mg: bool = False) -> float:
    """Bytes the method must move per launch of each kernel (no cache re-reads).

    rb: bytes of the real type; n: particles; cells: grid cells; faces: face
    counts per component; fluid: fluid cells of the solve; coarse: cells of the
    multigrid's coarse levels; mg: the multigrid solve with FP32 vectors, whose
    direction kernel also stores q = A s and whose update kernel also does the
    V-cycle's fine-level restriction (mg_down_fine then runs once per solve).
    """
    F = sum(faces)
    if mg and kind == "pcg_direction":
        return fluid * (4 * rb + 1)                     # z, s_old, diag in; s, q out
    if mg and kind == "pcg_update":
        return fluid * (6 * rb + 1) + cells / 8 * rb    # x, s, r, q, diag in; x, r, level-1 b out
    return {
        # multigrid V-cycle: fine level r, n_c in, level-1 b out (down); r, n_c,
        # level-1 x in, z out (up); each coarse cell b, n_c in and b out below
        # (down), b, n_c and x below in, x out (up)
        "mg_down_fine": fluid * (rb + 1) + cells / 8 * rb,
        "mg_up_fine": fluid * (2 * rb + 1) + cells / 8 * rb,
        "mg_coarse": coarse * (3 * rb + 2),
        "bin_keys": n * (3 * rb + 8) + 12 * cells,     # positions in; key, rank out; count fill + RMW
        "bin_scan": 8 * cells,                          # counts in, starts out
        "bin_scatter": 16 * n,                          # key, rank, start in; slot out
        "bin_gather": n * (12 * rb + 20),               # slot, key, start, count, state in; state out
        "tiles": 4 * cells,                             # counts in
        "p2g": n * 6 * rb + 8 * cells + 2 * rb * F,    # particles, hash in; raw and forced faces out
        "rhs": 3 * rb * F / 3 + fluid * (1 + 5 * rb),   # face differences in; diag, b, z, x, s out
        "pcg_direction": fluid * (3 * rb + 1),          # z, s_old, diag in; s out
        "pcg_update": fluid * (5 * rb + 1),             # x, s, z, diag in; x, z out
        "project": 2 * rb * F / 3 + 4 * cells + rb * fluid / 3,  # one component
        "g2p": n * 12 * rb + 6 * rb * F,                # particle state in/out; 6 face arrays in
    }[kind]


def traffic_for(kernel: str, scene: str):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary in
    profiles/ was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{scene}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2404_01931_amd", "csrc", vals.get("source", ""))
    if not os.path.exists(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if digest != vals.get("source_sha256"):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(sample_scene: str, steps: int):
    """Time the FP64 oracle (plain serial C) for a few steps of a bounded sample."""
    import numpy as np

    import oracle as O
    from paper_2404_01931_amd import inputs

    O.build(force=False)
    sc = inputs.scene(sample_scene)
    g = O.Grid(sc.n, sc.n, sc.n, sc.dx)
    regs = [O.Region(kind=r.kind, lo=r.lo, hi=r.hi, center=r.center, radius=r.radius, vel=r.vel)
            for r in sc.regions]
    pos, vel = O.seed(g, regs, sc.sub, sc.seed)
    pos = pos.astype(np.float32).astype(np.float64)
    prm = O.Params(grid=g, gravity=sc.gravity, dt=sc.dt, flip_ratio=sc.flip_ratio, density=sc.density,
                   tol=sc.tol)
    n = pos.shape[1]
    ids = None
    iters = []
    t0 = time.perf_counter()
    for _ in range(steps):
        res = O.step(prm, pos, vel, ids)
        pos, vel, ids = res.pos, res.vel, res.ids
        iters.append(res.solve.iterations)
    t = time.perf_counter() - t0
    return {
        "value": n * steps / t,
        "unit": "particle-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{steps} FP64 oracle step{'s' if steps != 1 else ''} (serial C, one thread, MIC(0)-PCG to "
                   f"{sc.tol:g}, {iters} iterations) of scene {sc.name} ({sc.n}^3, {n} particles) from its "
                   f"seeded start, {t:.1f} s; the value is particles x steps / time"),
        "host_cpu": host_cpu_model(),
        "host_nproc": os.cpu_count(),
        "threads": 1,
    }


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def serving_leg(n_scenes: int, budget_gib: float, slots: int, graphs: bool, plain_sample: int,
                multigrid: bool = True):
    """The batched-serving form: a stream of independent dam-break and drop
    scenes (sides 32/48/64/96, 8 particles per cell, 100 FP32 steps each at
    dt = 1/240, Poisson arrivals at 200 / s) through the continuous-batching
    server under an HBM budget, beside the plain path (flip_step, one scene at
    a time) on the first scenes of the same stream."""
    import torch

    from paper_2404_01931_amd import flip, inputs
    from paper_2404_01931_amd.serving import FlipBackend, Server, requests_from_scenes

    stream = inputs.serving_scenes(count=n_scenes)
    reqs = requests_from_scenes(stream)
    be = FlipBackend(graphs=graphs, multigrid=multigrid)
    cfg_flags = flip.FLIP_FLAG_MULTIGRID if multigrid else 0
    # warm the kernels and the graph path on two tiny requests
    warm = [(0.0, dataclasses.replace(sc, steps=3)) for _, sc in stream[:2]]
    Server(be, budget_bytes=2**34, max_slots=4).run(requests_from_scenes(warm))
    budget = int(budget_gib * 2**30)
    progress(f"serving: {n_scenes} scenes, budget {budget_gib} GiB, {slots} slots, graphs={graphs}")
    rep = Server(be, budget_bytes=budget, max_slots=slots).run(reqs)
    s = rep.summary()
    progress(f"serving: {s['completed']} scenes in {s['wall_s']:.2f} s, {s['particle_steps_per_s']:.3e} "
             f"particle-steps/s, step p50 {s['step_latency_ms_p50']:.2f} ms p99 {s['step_latency_ms_p99']:.2f} ms")
    # the plain path, one scene at a time, GPU stepping time only
    ps_plain, t_plain = 0, 0.0
    for _, sc in stream[:plain_sample]:
        cfg, keep = flip.scene_config(sc, flags=cfg_flags)
        sim = flip.Simulation(cfg, keep)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(sc.steps)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t
        ps_plain += sim.n * sc.steps
        sim.close()
    plain = ps_plain / t_plain if t_plain > 0 else None
    # the batched path on the same sample, all admitted at once
    sample = requests_from_scenes([(0.0, sc) for _, sc in stream[:plain_sample]])
    rep_b = Server(be, budget_bytes=2**38, max_slots=max(plain_sample, 1)).run(sample)
    sb = rep_b.summary()
    progress(f"serving: plain {plain:.3e} vs batched {sb['particle_steps_per_s']:.3e} particle-steps/s "
             f"on the first {plain_sample} scenes")
    return {
        "workload": f"{n_scenes} scenes of the serving stream (dam break / drop, sides 32-96, 8 ppc, "
                    f"100 FP32 steps, dt 1/240, Poisson arrivals 200/s, "
                    f"{'multigrid' if multigrid else 'Jacobi'}-PCG tol 1e-6)",
        "budget_GiB": budget_gib, "max_slots": slots, "graphs": graphs,
        **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()},
        "plain_sample_scenes": plain_sample,
        "plain_particle_steps_per_s": plain,
        "batched_sample_particle_steps_per_s": sb["particle_steps_per_s"],
    }


def surface_timing(sim, cfg, torch, reps: int = 5, refine: int = 1) -> dict:
    """Surface reconstruction on the handle's final state (Sec. 3.3): the
    improved-blobby field at the grid's corners (particle radius dx/2, search
    radius 2 dx; the call bins first) and marching cubes with vertex normals
    (the call reads its counts back), each timed with HIP events on the
    handle's stream over `reps` calls."""
    dx = cfg.dx
    st = sim.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    phi = sim.surface_field_device(0.5 * dx, 2 * dx, refine)
    mesh = sim.surface_mesh_device(phi, refine)
    st.synchronize()
    ev[0].record(st)
    for _ in range(reps):
        phi = sim.surface_field_device(0.5 * dx, 2 * dx, refine)
    ev[1].record(st)
    for _ in range(reps):
        mesh = sim.surface_mesh_device(phi, refine)
    ev[2].record(st)
    st.synchronize()
    out = {"corners": phi.numel(), "field_ms": round(ev[0].elapsed_time(ev[1]) / reps, 3),
           "mesh_ms": round(ev[1].elapsed_time(ev[2]) / reps, 3), "vertices": int(mesh[0].shape[0]),
           "triangles": int(mesh[2].shape[0]), "radius": "dx/2", "search": "2 dx", "refine": refine}
    progress(f"surface: {out}")
    return out


def surface_paper_workload(torch) -> dict:
    """The water drop of the paper's marching-cubes timings (about 300 k
    particles meshed on a 104^3 grid): a drop scene on a 52^3 simulation grid,
    10 steps in, field and mesh at refine 2 (104^3 sampling cells)."""
    import dataclasses

    from paper_2404_01931_amd import flip, inputs

    sc = dataclasses.replace(inputs.scene("drop64"), n=52, name="drop52")
    cfg, keep = flip.scene_config(sc, flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    sim.step(10)
    out = surface_timing(sim, cfg, torch, refine=2)
    out.update({"workload": f"drop52: {sim.n} particles, 52^3 simulation grid, 104^3 sampling grid, FP32"})
    sim.close()
    return out


def measure(args, sc, solver: str, with_surface: bool = False) -> dict:
    """Throughput of `args.steps` steps of scene sc on one handle (after
    `args.warmup`), then per-kernel durations on a second handle with kernel
    timing on. solver: "jacobi", "multigrid" (FLIP_FLAG_MULTIGRID) or "rbgs"
    (FLIP_FLAG_RED_BLACK_GS: the paper's red-black Gauss-Seidel instead of CG)."""
    import torch

    from paper_2404_01931_amd import flip

    mgflag = flip.FLIP_FLAG_MULTIGRID if solver == "multigrid" else 0
    sflag = mgflag | (flip.FLIP_FLAG_RED_BLACK_GS if solver == "rbgs" else 0)
    # reseeding adds particles: room for 6 per cell (the scenes seed fewer than 3 per cell)
    cap = 0
    if args.reseed:
        sflag |= flip.FLIP_FLAG_RESEED
        cap = 6 * sc.n**3
    # throughput: a handle without kernel timing (timed launches cost extra work)
    cfg, keep = flip.scene_config(sc, flags=sflag, capacity=cap)
    progress(f"init {sc.name} ({solver})")
    t = time.perf_counter()
    sim = flip.Simulation(cfg, keep)
    progress(f"init done in {time.perf_counter() - t:.1f} s: {sim.n} particles, workspace "
             f"{sim.ws_bytes / 2**30:.2f} GiB")
    if args.warmup:
        sim.step(args.warmup)
    s_pre = sim.stats()
    progress(f"warmup done ({args.warmup} steps, last {s_pre.pcg_iterations} PCG iterations)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.reseed:
        # the particle count grows: sum each step's count (a reseeding step
        # already waits for the device once, for its new total)
        particle_steps = 0
        for _ in range(args.steps):
            sim.step(1)
            particle_steps += sim.stats().n_particles
    else:
        sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    s_last = sim.stats()
    n = s_last.n_particles
    if not args.reseed:
        particle_steps = n * args.steps
    progress(f"timed {args.steps} steps in {elapsed:.3f} s")
    surface = surface_timing(sim, cfg, torch) if with_surface else None
    sim.close()
    del sim
    # kernel durations: a second handle of the same scene with kernel timing on
    # (HIP events; the solver kernels record their own start and end), stepped
    # through the same warm-up and a few more steps
    # (diagnostics on: the solve's true residual and the divergence left, in
    # FP64, by kernels outside the timed list)
    cfg_t, keep_t = flip.scene_config(sc, flags=flip.FLIP_FLAG_KERNEL_TIMING | flip.FLIP_FLAG_DIAGNOSTICS | sflag,
                                      capacity=cap)
    sim = flip.Simulation(cfg_t, keep_t)
    if args.warmup:
        sim.step(args.warmup)
    s0 = sim.stats()
    sim.step(args.timing_steps)
    s1 = sim.stats()
    progress(f"kernel timing over {args.timing_steps} steps")

    rb = 8 if cfg.precision == flip.FLIP_FP64 else 4
    fused = bool(mgflag) and rb == 4  # the FP32-vector multigrid solve fuses its update and fine restriction
    cells = cfg.nx * cfg.ny * cfg.nz
    faces = [(cfg.nx + 1) * cfg.ny * cfg.nz, cfg.nx * (cfg.ny + 1) * cfg.nz, cfg.nx * cfg.ny * (cfg.nz + 1)]
    d_iter = s1.pcg_iterations_total - s0.pcg_iterations_total
    d_cell_iter = s1.pcg_cell_iterations_total - s0.pcg_cell_iterations_total
    fluid_avg = d_cell_iter / d_iter if d_iter else 0.0
    kernels = {}
    for k, name in enumerate(flip.KERNEL_NAMES):
        cnt = s1.kernel_launches[k] - s0.kernel_launches[k]
        ms = s1.kernel_ms[k] - s0.kernel_ms[k]
        if cnt <= 0:
            continue
        avg = ms / cnt
        # the iteration kernels are timed on a sample of the iterations; the
        # fine restriction of the FP32 multigrid solve's first V-cycle (the
        # later ones are inside the update kernel) on every launch
        sampled = name.startswith(("pcg_", "mg_")) and not (fused and name == "mg_down_fine")
        launches = d_iter if sampled else cnt
        kernels[name] = {"avg_ms": avg, "launches": launches, "est_total_ms": avg * launches}
    ts = args.timing_steps
    # the dominant single kernel (mg_coarse times several launches together)
    dominant = max((k for k in kernels if k != "mg_coarse"), key=lambda k: kernels[k]["est_total_ms"])
    kd = kernels[dominant]
    coarse = mg_coarse_cells(cfg.nx, cfg.ny, cfg.nz) if mgflag else 0
    abytes = algorithmic_bytes(dominant, rb, n, cells, faces, fluid_avg, coarse, fused)
    achieved = abytes / (kd["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_for(dominant, sc.name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dominant,
                "avg_launch_ms": round(kd["avg_ms"], 5), "bytes_per_launch": abytes}
    pcg_ms = sum(v["est_total_ms"] for k, v in kernels.items() if k.startswith(("pcg_", "mg_")))
    pcg_bytes = d_cell_iter * (8 * rb + 2)
    if fused:
        # direction 4 rb + 1, update with the fine restriction 6 rb + 1, fine
        # prolongation 2 rb + 1 per fluid cell; level-1 b out and x in; the
        # coarse levels
        pcg_bytes = d_cell_iter * (12 * rb + 3) + d_iter * (cells / 4 * rb + coarse * (3 * rb + 2))
    elif mgflag:
        pcg_bytes += d_cell_iter * (3 * rb + 2) + d_iter * (cells / 4 * rb + coarse * (3 * rb + 2))
    pcg = {"iterations_per_step": (s_last.pcg_iterations_total - s_pre.pcg_iterations_total) / args.steps,
           "iterations_per_step_timing_run": d_iter / ts, "fluid_cells": round(fluid_avg),
           "last_residual_rel": s_last.max_r / s_last.max_b if s_last.max_b else 0.0,
           "refinements_last_step": s_last.refinements,
           "true_residual_fp64": s1.true_residual, "div_ratio_fp64": s1.div_ratio,
           "algorithmic_GBps": round(pcg_bytes / (pcg_ms * 1e-3) / 1e9, 1) if pcg_ms else None,
           "frac_of_hbm_peak": round(pcg_bytes / (pcg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if pcg_ms else None,
           "ms_per_step": round(pcg_ms / ts, 3)}
    stage_ms = {k: round(v["est_total_ms"] / ts, 3) for k, v in kernels.items()}
    progress(f"per-step kernel ms: {stage_ms}")

    sim.close()
    del sim
    return {"solver": solver, "n": n, "n0": s_pre.n_particles, "particle_steps": particle_steps,
            "elapsed": elapsed, "roofline": roofline, "pcg": pcg, "stage_ms": stage_ms, "surface": surface}


def precision_forms(args, headline: dict, sc) -> dict:
    """The mixed-precision solve (FP32 vectors, FP64 reductions and residual,
    iterative refinement to 1e-8) on the headline scene, against the plain FP64
    solve to the same tolerance and the plain FP32 solve, each timed on the GPU
    with its FP64 true residual and the divergence left after the projection."""
    from paper_2404_01931_amd import inputs

    def row(r, sc_r):
        return {"value": r["particle_steps"] / r["elapsed"], "unit": "particle-steps/s",
                "ms_per_step": r["elapsed"] / args.steps * 1e3,
                "tolerance": sc_r.ir_tol if sc_r.precision == "mixed" else sc_r.tol,
                "iterations_per_step": r["pcg"]["iterations_per_step"],
                "refinements_last_step": r["pcg"]["refinements_last_step"],
                "true_residual_fp64": r["pcg"]["true_residual_fp64"], "div_ratio_fp64": r["pcg"]["div_ratio_fp64"],
                "pcg_ms_per_step": r["pcg"]["ms_per_step"]}

    out = {"fp32": row(headline, sc)}
    mixed = inputs.scene(sc.name + "_mixed") if sc.name + "_mixed" in inputs.SCENES else \
        dataclasses.replace(sc, precision="mixed", tol=1e-4, ir_tol=1e-8)
    progress(f"precision forms: {mixed.name} mixed")
    out["mixed"] = row(measure(args, mixed, "multigrid"), mixed)
    fp64 = dataclasses.replace(sc, name=sc.name + "_fp64", precision="fp64", tol=mixed.ir_tol)
    progress(f"precision forms: {fp64.name} to {fp64.tol:g}")
    out["fp64_same_tolerance"] = row(measure(args, fp64, "multigrid"), fp64)
    out["note"] = ("mixed and fp64 solve to the same relative residual (1e-8); fp32 solves to 1e-6 on its "
                   "recursive residual, its FP64 true residual is what FP32 vectors allow")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scene", default="drop256")
    ap.add_argument("--precision", choices=["fp32", "fp64", "mixed"], default=None,
                    help="override the scene's precision")
    ap.add_argument("--cpu-sample", default="drop256")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--timing-steps", type=int, default=10,
                    help="steps of the separate handle that times each kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-scenes", type=int, default=512,
                    help="scenes of the serving stream to serve after the main benchmark (0: skip)")
    ap.add_argument("--serving-budget-gib", type=float, default=4.0)
    ap.add_argument("--serving-slots", type=int, default=128)
    ap.add_argument("--serving-no-graphs", action="store_true")
    ap.add_argument("--serving-plain-sample", type=int, default=16)
    ap.add_argument("--serving-only", action="store_true", help="skip the 256^3 benchmark")
    ap.add_argument("--solver", choices=["multigrid", "jacobi", "rbgs"], default="multigrid",
                    help="preconditioner of the pressure CG for the headline number (the other one is "
                         "measured too and reported beside it), or rbgs: the paper's red-black "
                         "Gauss-Seidel solver alone")
    ap.add_argument("--no-second-solver", action="store_true", help="measure the headline solver only")
    ap.add_argument("--no-surface", action="store_true", help="skip the surface reconstruction timing")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip the mixed-precision and FP64 solves of the headline scene")
    ap.add_argument("--reseed", action="store_true",
                    help="particle reseeding on (Sec. 3.1.2): sparse fluid cells are refilled each step")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scales HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        torch.cuda.set_device(0)
        n = args.calibrate_copy * 2**20 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the timestep has no multi-GPU "
              f"path in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2404_01931_amd import flip, inputs

    torch.cuda.set_device(0)
    if args.serving_only:
        out = serving_leg(args.serving_scenes, args.serving_budget_gib, args.serving_slots,
                          not args.serving_no_graphs, args.serving_plain_sample, args.solver == "multigrid")
        print(json.dumps({"serving": out}), flush=True)
        return
    sc = inputs.scene(args.scene)
    if args.precision:
        sc = inputs.scene(args.scene, precision=args.precision)
    # the headline solver, then the other one on the same scene for comparison
    solvers = ["jacobi", "multigrid"] if args.solver == "jacobi" else ["multigrid", "jacobi"]
    if args.solver == "rbgs":
        solvers = ["rbgs"]
    if args.no_second_solver:
        solvers = solvers[:1]
    runs = {name: measure(args, sc, name, with_surface=(name == solvers[0] and not args.no_surface))
            for name in solvers}
    main_run = runs[solvers[0]]
    forms = None
    if not args.no_precision_forms and sc.precision == "fp32" and main_run["solver"] == "multigrid":
        forms = precision_forms(args, main_run, sc)
    serving = None
    if args.serving_scenes > 0:
        serving = serving_leg(args.serving_scenes, args.serving_budget_gib, args.serving_slots,
                              not args.serving_no_graphs, args.serving_plain_sample, args.solver == "multigrid")

    cpu = None
    if not args.no_cpu_baseline:
        progress(f"cpu baseline: oracle on {args.cpu_sample}")
        cpu = cpu_baseline(args.cpu_sample, args.cpu_steps)
        progress(f"cpu baseline: {cpu['value']:.3e} particle-steps/s")

    n, elapsed = main_run["n"], main_run["elapsed"]
    solver_label = {"jacobi": "Jacobi-PCG", "multigrid": "multigrid-PCG", "rbgs": "red-black Gauss-Seidel"}
    line = {
        "metric": "particle-steps/s",
        "value": main_run["particle_steps"] / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "mixed": "f32+f64"}[sc.precision],
        "data": "synthetic",
        "config": {"workload": f"{sc.name}: {inputs.describe(sc)}, {sc.n}^3 MAC grid, {n} particles, "
                               f"{sc.precision.upper()}, dt=1/{round(1 / sc.dt)}, FLIP {sc.flip_ratio}, "
                               f"{solver_label[main_run['solver']]} tol {sc.tol:g}"
                               + (f", FP64 refinement to {sc.ir_tol:g}" if sc.precision == "mixed" else "")
                               + (f", particle reseeding ({main_run['n0']} particles after warmup)"
                                  if args.reseed else ""),
                   "grid": sc.n, "particles": n, "parallelism": "single GPU"},
        "roofline": main_run["roofline"],
        "pcg": main_run["pcg"],
        "kernel_ms_per_step": main_run["stage_ms"],
    }
    for name, r in runs.items():
        if r is main_run:
            continue
        line[f"{name}_pcg_same_scene"] = {
            "value": r["particle_steps"] / r["elapsed"], "unit": "particle-steps/s",
            "ms_per_step": r["elapsed"] / args.steps * 1e3, "roofline": r["roofline"], "pcg": r["pcg"],
            "kernel_ms_per_step": r["stage_ms"]}
    line["surface"] = main_run["surface"]
    if line["surface"] is not None:
        line["surface"]["paper_mc_workload"] = surface_paper_workload(torch)
    line["precision_forms"] = forms
    line["serving"] = serving
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
