"""Parity at the configured sizes, in the configuration the benchmark times.

- drop 256^3, FP32, multigrid-preconditioned CG (the headline scene, 42.3 M
  particles): after two warm-up steps, one step shadowed by the oracle from
  the GPU's state. Binning bit-exact; every stage against the oracle fed the
  GPU's own inputs (the whole grid and every particle); the solve's true
  residual evaluated in FP64 by the oracle's operator; the whole step against
  the oracle's step with a tight solve (velocities within 1e-4 relative,
  norm-wise and per particle). This exercises the solver kernels' launch
  shapes that only grids of 128^3 and up use (the 512-thread coarse levels).
- dam break 128^3, FP32, multigrid: four steps, each shadowed by the oracle's
  full step.
- drop 256^3, mixed precision with multigrid inner solves: the FP64 true
  residual of the solution, evaluated by the oracle, meets the 1e-8
  refinement tolerance.
The oracle's solve at 256^3 takes one to two minutes of one host core.
"""
import numpy as np
import pytest

import oracle as O
from paper_2404_01931_amd import flip, inputs
from tests.gpu_util import grid_of, l2_rel, log, max_rel, params_of, state
from tests.test_gpu_parity import U32, fp32_true_residual_bound

pytestmark = pytest.mark.gpu

FP32_TOL = 2e-5  # stage agreement in FP32 on identical inputs (as in test_gpu_parity.py)


def _f64(fs):
    return [np.asarray(f, np.float64) for f in fs]


@pytest.mark.timeout(1200)
def test_drop256_fp32_multigrid_step_matches_oracle(orc):
    sc = inputs.scene("drop256")
    log("[fullsize] drop256 init")
    cfg, keep = flip.scene_config(sc, flags=flip.FLIP_FLAG_MULTIGRID | flip.FLIP_FLAG_DIAGNOSTICS)
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    pos0, vel0, ids0 = state(sim)
    sim.step(1)
    st = sim.stats()
    g = grid_of(sim)
    prm = params_of(sim, tol=1e-9)
    log(f"[fullsize] drop256: n={pos0.shape[1]} iters={st.pcg_iterations} fluid={st.n_fluid_cells}")
    assert st.pcg_status == 0

    # binning, bit for bit
    key, count, start, perm = O.bin_particles(g, pos0)
    fluid = O.fluid_flags(g, count)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), count)
    assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_START), start)
    ids = sim.read(flip.FLIP_FIELD_ID)
    assert np.array_equal(ids, ids0[perm])
    del key
    pos_s, vel_s = np.ascontiguousarray(pos0[:, perm]), np.ascontiguousarray(vel0[:, perm])
    log("[fullsize] drop256: binning bit-exact")

    # particle-to-grid, forces, right-hand side on the GPU's inputs
    u_old = _f64(sim.faces(flip.FLIP_FIELD_U_OLD))
    ref_old, wts = O.p2g(g, pos_s, vel_s, return_weights=True)
    vmax = np.abs(vel_s).max()
    for a in range(3):
        ok = wts[a] >= 1e-3
        assert max_rel(u_old[a][ok], ref_old[a][ok]) <= FP32_TOL
        assert np.all(np.abs(u_old[a][~ok]) <= vmax * (1 + 1e-6))
    del ref_old, wts
    u_star = _f64(sim.faces(flip.FLIP_FIELD_U_STAR))
    ref_star = O.forces_walls(g, u_old, prm.gravity, prm.dt)
    for a in range(3):
        assert max_rel(u_star[a], ref_star[a]) <= FP32_TOL
    del ref_star
    b = sim.read(flip.FLIP_FIELD_RHS).astype(np.float64)
    b_ref = O.rhs(g, fluid, u_star, prm.density, prm.dt)
    assert max_rel(b, b_ref) <= 10 * FP32_TOL
    del b_ref
    log("[fullsize] drop256: particle-to-grid, forces and right-hand side agree")

    # the solve: the FP32 pressure against its own system, in FP64
    p = sim.read(flip.FLIP_FIELD_PRESSURE).astype(np.float64)
    assert np.all(p[fluid == 0] == 0)
    true_rel = np.abs(b - orc.apply_A(g, fluid, p)).max() / np.abs(b).max()
    bound = fp32_true_residual_bound(st.pcg_iterations, p, b, cfg.pcg_tol)
    log(f"[fullsize] drop256: true residual {true_rel:.3e} (bound {bound:.3e}, library {st.true_residual:.3e})")
    assert st.max_r <= cfg.pcg_tol * st.max_b * (1 + 1e-12)
    assert true_rel <= bound
    assert abs(st.true_residual - true_rel) <= 1e-13 * (1 + 12 * np.abs(p).max() / np.abs(b).max())

    # projection with the GPU's pressure; divergence left
    u_new = _f64(sim.faces(flip.FLIP_FIELD_U_NEW))
    ref_new = O.project(g, fluid, p, prm.density, prm.dt, u_star)
    for a in range(3):
        assert max_rel(u_new[a], ref_new[a]) <= 10 * FP32_TOL
    del ref_new
    div_new = orc.divergence(g, u_new)[fluid == 1]
    div_star = orc.divergence(g, u_star)[fluid == 1]
    ratio = np.abs(div_new).max() / np.abs(div_star).max()
    umax = max(np.abs(np.concatenate(u_new)).max(), np.abs(np.concatenate(u_star)).max())
    log(f"[fullsize] drop256: divergence ratio {ratio:.3e} (library {st.div_ratio:.3e})")
    assert ratio <= 1.01 * true_rel + 12 * U32 * umax / (g.dx * np.abs(div_star).max())
    assert st.div_ratio == pytest.approx(ratio, rel=1e-12)
    del div_new, div_star

    # grid-to-particle on the GPU's grids, every particle
    pos1, vel1, _ = state(sim)
    ref_pos, ref_vel = O.g2p_advect(g, pos_s, vel_s, u_new, u_old, prm.flip_ratio, prm.dt)
    assert max_rel(vel1, ref_vel) <= 10 * FP32_TOL
    assert np.abs(pos1 - ref_pos).max() <= 2e-6
    del ref_pos, ref_vel
    sim.close()
    log("[fullsize] drop256: projection and grid-to-particle agree; oracle step (tight solve) ...")

    # the whole step against the oracle's step with a tight solve
    res = orc.step(prm, pos0, vel0, ids0)
    assert np.array_equal(res.ids, ids)
    ev, ep = l2_rel(vel1, res.vel), max_rel(vel1, res.vel)
    log(f"[fullsize] drop256: oracle solve {res.solve.iterations} iterations; step velocity error l2 {ev:.3e} "
        f"max {ep:.3e}; pos max {np.abs(pos1 - res.pos).max():.3e}")
    assert ev <= 1e-4
    assert ep <= 1e-4


@pytest.mark.timeout(600)
def test_dam128_fp32_multigrid_shadowed_steps(orc):
    sc = inputs.scene("dam128")
    log("[fullsize] dam128 init")
    cfg, keep = flip.scene_config(sc, flags=flip.FLIP_FLAG_MULTIGRID)
    sim = flip.Simulation(cfg, keep)
    prm = params_of(sim)
    for s in range(4):
        pos0, vel0, ids0 = state(sim)
        sim.step(1)
        pos1, vel1, ids1 = state(sim)
        res = orc.step(prm, pos0, vel0, ids0)
        assert np.array_equal(res.ids, ids1)
        assert np.array_equal(sim.read(flip.FLIP_FIELD_CELL_COUNT), res.count)
        ev, ep = l2_rel(vel1, res.vel), max_rel(vel1, res.vel)
        log(f"[fullsize] dam128 step {s}: iters {sim.stats().pcg_iterations}, velocity error l2 {ev:.3e} "
            f"max {ep:.3e}")
        assert ev <= 1e-4 and ep <= 1e-4
        assert np.abs(pos1 - res.pos).max() <= 1e-4
    sim.close()


@pytest.mark.timeout(600)
def test_drop256_mixed_true_residual(orc):
    sc = inputs.scene("drop256_mixed")
    log("[fullsize] drop256 mixed init")
    cfg, keep = flip.scene_config(sc, flags=flip.FLIP_FLAG_MULTIGRID | flip.FLIP_FLAG_DIAGNOSTICS)
    sim = flip.Simulation(cfg, keep)
    sim.step(2)
    st = sim.stats()
    g = grid_of(sim)
    count = sim.read(flip.FLIP_FIELD_CELL_COUNT)
    fluid = O.fluid_flags(g, count)
    b = sim.read(flip.FLIP_FIELD_RHS)
    p = sim.read(flip.FLIP_FIELD_PRESSURE)
    assert b.dtype == np.float64 and p.dtype == np.float64
    true_rel = np.abs(b - orc.apply_A(g, fluid, p)).max() / np.abs(b).max()
    log(f"[fullsize] drop256 mixed: {st.pcg_iterations} inner iterations, {st.refinements} refinements, "
        f"true residual {true_rel:.3e} (library {st.true_residual:.3e}), divergence ratio {st.div_ratio:.3e}")
    assert st.pcg_status == 0
    assert true_rel <= 1.01 * cfg.ir_tol
    # two FP64 evaluations of the same residual differ by their rounding: each
    # r_c = b_c - (n_c p_c - sum p_nb) is a sum of 8 terms of size up to max|b|
    # and 12 max|p| (as in the FP32 test)
    assert abs(st.true_residual - true_rel) <= 1e-13 * (1 + 12 * np.abs(p).max() / np.abs(b).max())
    sim.close()
