"""GPU parity: each stage of one HIP timestep, called through the C ABI, against
the FP64 oracle fed the GPU's own inputs; then the whole step against the
oracle's step (exact solve) from the same state.

Tolerances: integer work (keys, counts, scan, permutation, flags) is compared
bit for bit. Floating-point stages fed identical inputs must agree to the
rounding of the GPU's precision: 2e-5 relative (FP32, sums of ~64 hat-weighted
terms) or 1e-11 (FP64). The whole step must keep particle velocities within
1e-4 relative of the oracle's, norm-wise and for the largest single deviation.

The FP32 solve stops on its recursive residual; its true residual, evaluated
in FP64, is gated by the residual-gap bound of CG in finite precision: after k
iterations the true and the recursive residual differ by at most about
k u (max|b| + |A| max|p|) with u = 2^-24 and |A| <= 12 (n_c <= 6 plus six
neighbours), so true/max|b| <= tol + 2 k u (1 + 12 max|p| / max|b|). The FP32
divergence ratio adds the rounding of the stored faces to that: each divergence
sums six differences of FP32 faces, 12 u max|u| / dx at most. FP64 and the
mixed path (test_gpu_mixed.py) meet 1e-6 on the true residual itself.
"""

U32 = 2.0 ** -24


def fp32_true_residual_bound(iters, p, b, tol):
    """Residual-gap bound of an FP32 CG solve (see the module docstring)."""
    mb = np.abs(b).max()
    return tol + 2 * max(iters, 1) * U32 * (1 + 12 * np.abs(p).max() / mb)
import numpy as np
import pytest

import oracle as O
from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import by_id, grid_of, l2_rel, log, max_rel, params_of, state

pytestmark = pytest.mark.gpu


def _ragged_case(prec):
    # 20 x 12 x 17 cells: tiles overhang the domain on every axis
    shape, dx = (20, 12, 17), 1.0 / 20
    L = np.array(shape) * dx
    pos, vel = inputs.random_particles(shape, 9000, seed=21, lo=(0.0, 0.0, 0.0), hi=(0.55, 0.4, L[2]), dx=dx)
    # a few particles on cell planes and in the same spot (ties)
    pos[:, :50] = np.round(pos[:, :50] / dx) * dx
    pos[:, 50:80] = pos[:, 80:110]
    # inside the domain also after rounding to the working precision
    pos = np.clip(pos, 0.0, L[:, None] * (1 - 1e-6))
    if prec == flip.FLIP_FP32:
        pos = pos.astype(np.float32).astype(np.float64)
        vel = vel.astype(np.float32).astype(np.float64)
    cfg, keep = flip.make_config(shape, dx, 1 / 240, precision=prec, pcg_tol=1e-6, pos0=pos, vel0=0.5 * vel)
    return cfg, keep


def make_case(name):
    if name == "dam32_fp64":
        return flip.scene_config(inputs.scene("dam32"))
    if name == "dam32_fp32":
        return flip.scene_config(inputs.scene("dam32"), precision=flip.FLIP_FP32)
    if name == "ragged_fp32":
        return _ragged_case(flip.FLIP_FP32)
    if name == "ragged_fp64":
        return _ragged_case(flip.FLIP_FP64)
    if name == "drop64_fp32":
        return flip.scene_config(inputs.scene("drop64"))
    if name == "ddam32_fp64":
        return flip.scene_config(inputs.scene("ddam32"))
    raise KeyError(name)


CASES = ["dam32_fp64", "dam32_fp32", "ragged_fp32", "ragged_fp64", "drop64_fp32", "ddam32_fp64"]


def _tol(sim):
    return 1e-11 if sim.cfg.precision == flip.FLIP_FP64 else 2e-5


def _f64(fs):
    return [np.asarray(f, np.float64) for f in fs]


@pytest.mark.parametrize("case", CASES)
def test_seeded_or_uploaded_state_matches_oracle(orc, case):
    log(f"[parity] init {case}")
    cfg, keep = make_case(case)
    sim = flip.Simulation(cfg, keep)
    pos, vel, ids = state(sim)
    assert np.array_equal(ids, np.arange(pos.shape[1], dtype=np.uint32))
    if cfg.pos0:
        return
    sc = {"dam32_fp64": "dam32", "dam32_fp32": "dam32", "drop64_fp32": "drop64", "ddam32_fp64": "ddam32"}[case]
    s = inputs.scene(sc)
    from tests.scenes_util import oracle_grid, oracle_regions

    p_ref, v_ref = orc.seed(oracle_grid(s), oracle_regions(s), s.sub, s.seed)
    p_ref = p_ref.astype(sim.real).astype(np.float64)
    v_ref = v_ref.astype(sim.real).astype(np.float64)
    assert np.array_equal(pos, p_ref)  # bitwise
    assert np.array_equal(vel, v_ref)
    sim.close()


@pytest.mark.parametrize("case", CASES)
def test_one_step_stage_parity(orc, case):
    log(f"[parity] one step {case}")
    cfg, keep = make_case(case)
    cfg.flags |= flip.FLIP_FLAG_DIAGNOSTICS
    sim = flip.Simulation(cfg, keep)
    g = grid_of(sim)
    tol = _tol(sim)
    pos0, vel0, ids0 = state(sim)
    sim.step(1)
    st = sim.stats()
    log(f"[parity] {case}: n={pos0.shape[1]} iters={st.pcg_iterations} fluid={st.n_fluid_cells} "
        f"tiles={st.n_active_tiles}")

    # binning: bit-exact
    key, count, start, perm = O.bin_particles(g, pos0)
    fluid = O.fluid_flags(g, count)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), count)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_START), start)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_FLAGS), fluid)
    ids = sim.read(flip.FLIP_FIELD_ID)
    assert np.array_equal(ids, ids0[perm])
    assert st.n_fluid_cells == int(fluid.sum())
    pos_s, vel_s = pos0[:, perm], vel0[:, perm]

    # particle-to-grid on the binned particles. A face whose total hat weight
    # is a rounding-level graze (a particle exactly one cell width away) has an
    # ill-conditioned value M/W; no particle reads it with more than that
    # weight, so such faces are only checked for being bounded.
    u_old = _f64(sim.faces(flip.FLIP_FIELD_U_OLD))
    ref_old, wts = O.p2g(g, pos_s, vel_s, return_weights=True)
    wmin = 1e-9 if sim.cfg.precision == flip.FLIP_FP64 else 1e-3
    vmax = np.abs(vel_s).max()
    for a in range(3):
        ok = wts[a] >= wmin
        assert max_rel(u_old[a][ok], ref_old[a][ok]) <= tol, ("p2g", a, max_rel(u_old[a][ok], ref_old[a][ok]))
        assert np.all(np.abs(u_old[a][~ok]) <= vmax * (1 + 1e-6))

    # gravity + walls on the GPU's raw transfer
    u_star = _f64(sim.faces(flip.FLIP_FIELD_U_STAR))
    prm = params_of(sim)
    ref_star = O.forces_walls(g, u_old, prm.gravity, prm.dt)
    for a in range(3):
        assert max_rel(u_star[a], ref_star[a]) <= tol, ("forces", a)

    # right-hand side from the GPU's u*
    b = sim.read(flip.FLIP_FIELD_RHS).astype(np.float64)
    b_ref = O.rhs(g, fluid, u_star, prm.density, prm.dt)
    assert max_rel(b, b_ref) <= 10 * tol
    assert st.max_b == pytest.approx(np.abs(b).max(), rel=1e-12)

    # solve: the GPU pressure must satisfy its own system to the solver tolerance
    p = sim.read(flip.FLIP_FIELD_PRESSURE).astype(np.float64)
    assert np.all(p[fluid == 0] == 0)
    assert st.pcg_status == 0
    r_true = b - orc.apply_A(g, fluid, p)
    true_rel = np.abs(r_true).max() / np.abs(b).max()
    log(f"[parity] {case}: true residual {true_rel:.3e} (solver's own {st.max_r / st.max_b:.3e})")
    assert st.max_r <= cfg.pcg_tol * st.max_b * (1 + 1e-12)
    fp64 = sim.cfg.precision == flip.FLIP_FP64
    bound = 1.01e-6 if fp64 else fp32_true_residual_bound(st.pcg_iterations, p, b, cfg.pcg_tol)
    log(f"[parity] {case}: true residual bound {bound:.3e}")
    assert true_rel <= bound
    # the library's own FP64 evaluation of the same residual (diagnostics)
    assert abs(st.true_residual - true_rel) <= 1e-13 * (1 + 12 * np.abs(p).max() / np.abs(b).max())
    exact = orc.pcg(g, fluid, b, 1e-13, 100000)
    dp = np.abs(p - exact.p).max()
    log(f"[parity] {case}: |p - p_exact| / |p_exact| = {l2_rel(p, exact.p):.3e}, max {dp:.3e}")

    # projection with the GPU's pressure
    u_new = _f64(sim.faces(flip.FLIP_FIELD_U_NEW))
    ref_new = O.project(g, fluid, p, prm.density, prm.dt, u_star)
    for a in range(3):
        assert max_rel(u_new[a], ref_new[a]) <= 10 * tol, ("project", a, max_rel(u_new[a], ref_new[a]))

    # grid-to-particle + advection on the GPU's grids
    pos1, vel1, _ = state(sim)
    ref_pos, ref_vel = O.g2p_advect(g, pos_s, vel_s, u_new, u_old, prm.flip_ratio, prm.dt)
    assert max_rel(vel1, ref_vel) <= 10 * tol, max_rel(vel1, ref_vel)
    assert np.abs(pos1 - ref_pos).max() <= (1e-13 if tol < 1e-9 else 2e-6)

    # whole step against the oracle's step with an exact solve
    res = orc.step(prm, pos0, vel0, ids0)
    assert np.array_equal(res.ids, ids)
    ev, ep = l2_rel(vel1, res.vel), max_rel(vel1, res.vel)
    log(f"[parity] {case}: step velocity error l2 {ev:.3e} max {ep:.3e}, "
        f"pos max {np.abs(pos1 - res.pos).max():.3e}")
    # norm-wise and largest single-particle relative velocity error against
    # the exact-solve step
    assert ev <= 1e-4
    assert ep <= 1e-4
    # derived per-particle bound: v = (1 - alpha) PIC + alpha (v + interp(u_new - u_old)),
    # interpolation a convex combination, so |dv| <= max|d u_new| + max|d u_old|, and
    # by Eq. (5) |d u_new| <= |d u*| + (dt / (rho dx)) 2 max|p - p_ref|
    dp_ref = np.abs(p - res.solve.p).max()
    du_old = max(np.abs(u_old[a] - res.u_old[a]).max() for a in range(3))
    du_star = max(np.abs(u_star[a] - res.u_star[a]).max() for a in range(3))
    dv_bound = 2 * prm.dt / (prm.density * g.dx) * dp_ref + du_star + du_old + 4 * tol * np.abs(res.vel).max()
    log(f"[parity] {case}: max|dv| {np.abs(vel1 - res.vel).max():.3e} <= derived {dv_bound:.3e} "
        f"(max|p - p_ref| {dp_ref:.3e})")
    assert np.abs(vel1 - res.vel).max() <= dv_bound
    # divergence after projection (relative to before), evaluated in FP64
    div_all = orc.divergence(g, u_new)
    div_new = div_all[fluid == 1]
    div_star = orc.divergence(g, u_star)[fluid == 1]
    ratio = np.abs(div_new).max() / np.abs(div_star).max()
    log(f"[parity] {case}: max|div u_new| / max|div u*| = {ratio:.3e}")
    if fp64:
        assert ratio <= 1.01e-6
    else:
        umax = max(np.abs(np.concatenate(u_new)).max(), np.abs(np.concatenate(u_star)).max())
        assert ratio <= 1.01 * true_rel + 12 * U32 * umax / (g.dx * np.abs(div_star).max())
    # the library's own FP64 divergence (diagnostics and the DIV field)
    assert st.div_ratio == pytest.approx(ratio, rel=1e-12)
    div_gpu = sim.read(flip.FLIP_FIELD_DIV)
    assert np.all(div_gpu[fluid == 0] == 0)
    assert np.abs(div_gpu[fluid == 1] - div_new).max() <= 1e-12 * np.abs(div_star).max()
    # particles' energy and speed after the step
    ke = 0.5 * float(np.sum(vel1 * vel1))
    assert st.kinetic_energy == pytest.approx(ke, rel=1e-12)
    assert st.max_speed == pytest.approx(float(np.sqrt((vel1 * vel1).sum(axis=0)).max()), rel=1e-12)
    assert st.cfl_number == pytest.approx(st.max_speed * prm.dt / g.dx, rel=1e-12)
    assert st.nonfinite == 0
    sim.close()


@pytest.mark.parametrize("case,steps", [("dam32_fp64", 20), ("dam32_fp32", 10), ("drop64_fp32", 5)])
def test_shadowed_multi_step_parity(orc, case, steps):
    """Every step, the oracle restarts from the GPU's state (one-step shadowing)."""
    log(f"[parity] shadow {case} x{steps}")
    cfg, keep = make_case(case)
    sim = flip.Simulation(cfg, keep)
    prm = params_of(sim)
    worst = 0.0
    for s in range(steps):
        pos0, vel0, ids0 = state(sim)
        sim.step(1)
        pos1, vel1, ids1 = state(sim)
        res = orc.step(prm, pos0, vel0, ids0)
        assert np.array_equal(res.ids, ids1)
        e = l2_rel(vel1, res.vel)
        worst = max(worst, e)
        assert e <= 1e-4, (s, e)
        assert np.abs(pos1 - res.pos).max() <= 1e-4 * g_len(sim)
    log(f"[parity] shadow {case}: worst velocity l2 error {worst:.3e}")
    sim.close()


def g_len(sim):
    return max(sim.shape) * sim.cfg.dx


def test_uniform_power_of_two_velocity_round_trip_is_bit_exact():
    log("[parity] uniform transfer")
    shape, dx, dt = (16, 16, 16), 1 / 16, 1 / 240
    pos, _ = inputs.random_particles(shape, 6000, seed=3, lo=(4 / 16,) * 3, hi=(12 / 16,) * 3, dx=dx)
    pos = pos.astype(np.float32).astype(np.float64)
    U = np.array([0.5, -2.0, 0.25])
    vel = np.repeat(U[:, None], pos.shape[1], axis=1)
    cfg, keep = flip.make_config(shape, dx, dt, precision=flip.FLIP_FP32, pos0=pos, vel0=vel,
                                 flags=flip.FLIP_FLAG_NO_GRAVITY | flip.FLIP_FLAG_NO_PROJECTION)
    sim = flip.Simulation(cfg, keep)
    sim.step(1)
    p1 = sim.read(flip.FLIP_FIELD_POS)
    v1 = sim.read(flip.FLIP_FIELD_VEL)
    ids = sim.read(flip.FLIP_FIELD_ID)
    assert np.all(v1 == U.astype(np.float32)[:, None])
    u_old = sim.faces(flip.FLIP_FIELD_U_OLD)
    for a in range(3):
        vals = np.unique(u_old[a])
        assert set(vals.tolist()) <= {0.0, float(np.float32(U[a]))}, (a, vals[:8])
    expect = pos.astype(np.float32)[:, ids] + (np.float32(dt) * U.astype(np.float32))[:, None]
    bad = np.flatnonzero((p1 != expect).any(axis=0))
    assert bad.size == 0, (bad.size, p1[:, bad[:3]], expect[:, bad[:3]])
    sim.close()


def test_hydrostatic_pool_stays_at_rest(orc):
    log("[parity] hydrostatic")
    n, J = 32, 10
    sc = inputs.Scene(name="pool", n=n, regions=(inputs.RegionSpec("box", hi=(9, J / n, 9)),), seed=9,
                      precision="fp32", dt=1 / 240, flip_ratio=0.95, tol=1e-6, steps=1)
    cfg, keep = flip.scene_config(sc)
    sim = flip.Simulation(cfg, keep)
    sim.step(1)
    g = grid_of(sim)
    p = sim.read(flip.FLIP_FIELD_PRESSURE).astype(np.float64)
    fl = sim.read(flip.FLIP_FIELD_FLAGS) == 1
    jj = (np.arange(g.ncells) // n) % n
    expected = 9.81 * g.dx * (J - jj)
    assert max_rel(p[fl], expected[fl]) <= 1e-4
    v = sim.read(flip.FLIP_FIELD_VEL)
    assert np.abs(v).max() <= 1e-4 * 9.81 / 240 * 10
    sim.close()


def test_ballistic_first_step_has_zero_rhs():
    log("[parity] ballistic")
    sc = inputs.Scene(name="blob", n=32, regions=(inputs.RegionSpec("sphere", center=(0.5, 0.5, 0.5), radius=0.15,
                                                                    vel=(0.5, 0.25, -0.5)),),
                      seed=4, precision="fp32", dt=1 / 256, flip_ratio=0.95, tol=1e-6, steps=1,
                      gravity=(0.0, -8.0, 0.0))
    cfg, keep = flip.scene_config(sc)
    sim = flip.Simulation(cfg, keep)
    sim.step(1)
    st = sim.stats()
    assert st.max_b == 0.0 and st.pcg_iterations == 0 and st.pcg_status == 0
    v = sim.read(flip.FLIP_FIELD_VEL)
    np.testing.assert_array_equal(v[1], np.float32(0.25 - 8.0 / 256))
    np.testing.assert_array_equal(v[0], np.float32(0.5))
    sim.close()


def test_empty_and_single_particle_and_one_cell_pileup(orc):
    log("[parity] degenerate inputs")
    # no particles at all
    cfg, keep = flip.make_config((8, 8, 8), 1 / 8, 1 / 240, pos0=np.zeros((3, 0)), vel0=np.zeros((3, 0)))
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    st = sim.stats()
    assert st.n_particles == 0 and st.n_active_tiles == 0 and st.pcg_iterations == 0
    assert np.all(sim.read(flip.FLIP_FIELD_CELL_COUNT) == 0)
    sim.close()
    # one particle
    cfg, keep = flip.make_config((8, 8, 8), 1 / 8, 1 / 240, pos0=np.array([[0.3], [0.6], [0.2]]),
                                 vel0=np.array([[0.1], [0.0], [-0.2]]))
    sim = flip.Simulation(cfg, keep)
    p0, v0, i0 = state(sim)
    sim.step(1)
    p1, v1, _ = state(sim)
    res = orc.step(params_of(sim), p0, v0, i0)
    assert l2_rel(v1, res.vel) <= 1e-4
    sim.close()
    # 3000 particles piled into one cell (long segment in the stable sort)
    rng = np.random.default_rng(8)
    pos = (np.array([[3.0], [2.0], [5.0]]) + rng.random((3, 3000))) / 8
    pos = pos.astype(np.float32).astype(np.float64)
    vel = rng.standard_normal((3, 3000)).astype(np.float32).astype(np.float64)
    cfg, keep = flip.make_config((8, 8, 8), 1 / 8, 1 / 240, pos0=pos, vel0=vel)
    sim = flip.Simulation(cfg, keep)
    p0, v0, i0 = state(sim)
    sim.step(1)
    g = grid_of(sim)
    key, count, start, perm = O.bin_particles(g, p0)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_ID), i0[perm])
    p1, v1, _ = state(sim)
    res = orc.step(params_of(sim), p0, v0, i0)
    assert l2_rel(v1, res.vel) <= 1e-4
    sim.close()


def test_two_runs_are_bitwise_identical():
    log("[parity] determinism")
    outs = []
    for _ in range(2):
        cfg, keep = flip.scene_config(inputs.scene("drop64"))
        sim = flip.Simulation(cfg, keep)
        sim.step(3)
        outs.append((sim.read(flip.FLIP_FIELD_POS), sim.read(flip.FLIP_FIELD_VEL), sim.read(flip.FLIP_FIELD_ID),
                     sim.read(flip.FLIP_FIELD_PRESSURE)))
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_not_converged_is_reported_and_latched():
    log("[parity] max iters")
    cfg, keep = flip.scene_config(inputs.scene("dam32"), pcg_max_iters=2)
    sim = flip.Simulation(cfg, keep)
    status = sim.step(1, allow=(flip.FLIP_E_NOT_CONVERGED,))
    assert status == flip.FLIP_E_NOT_CONVERGED
    st = sim.stats()
    assert st.pcg_iterations == 2 and st.pcg_status == 1
    assert st.latched_status == flip.FLIP_E_NOT_CONVERGED
    sim.close()
