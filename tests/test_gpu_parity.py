"""HIP step vs the CPU oracle, through the C ABI (needs an MI355X).

Every comparison starts both sides from the same float32 state read back from
the GPU, runs one step, and checks the integer outputs bit-exactly and the
float outputs against the tolerances in ``tests/parity.py``.
"""
import numpy as np
import pytest

import oracle
import paper_2311_15088_amd as sph
from paper_2311_15088_amd import scenes

from parity import compare_step, oracle_given_rho

pytestmark = pytest.mark.gpu


def gpu_fields(sim, diag=True):
    d = dict(key=sim.read(sph.CELL_KEY), off=sim.read(sph.CELL_OFFSETS), sorted=sim.read(sph.SORTED_IDS),
             nbr=sim.read(sph.NBR_COUNT), rho=sim.read(sph.DENSITY), x1=sim.read(sph.POS), v1=sim.read(sph.VEL),
             akey=sim.read(sph.AGENT_KEY), aoff=sim.read(sph.AGENT_CELL_OFFSETS),
             asorted=sim.read(sph.AGENT_SORTED_IDS), y1=sim.read(sph.AGENT_POS), u1=sim.read(sph.AGENT_VEL))
    if diag:
        d.update(a_int=sim.read(sph.ACC_INT), a_coup=sim.read(sph.ACC_COUPLE), touched=sim.read(sph.TOUCHED),
                 force=sim.read(sph.AGENT_FORCE), steer=sim.read(sph.AGENT_STEER), acounts=sim.read(sph.AGENT_COUNTS))
    return d


def state(sim):
    return sim.read(sph.POS), sim.read(sph.VEL), sim.read(sph.AGENT_POS), sim.read(sph.AGENT_VEL)


def chained_parity(sc, steps, fs=None, as_=None, nbr_mode=0, search=sph.SEARCH_TILES):
    print(f"[parity] scene {sc.name} n={sc.n} a={sc.n_agents} steps={steps} search={search}", flush=True)
    sim = sph.create(sc, flags=sph.FLAG_DIAGNOSTICS)
    if search != sph.SEARCH_TILES:
        sim.set_search(search)
    x, v, y, u = sc.x, sc.v, sc.y, sc.u
    worst = {}
    for k in range(steps):
        sim.step(1)
        g = gpu_fields(sim)
        ref = oracle.step(sc.params, x, v, y, u, fsample=fs, asample=as_, nbr_mode=nbr_mode)
        refc = oracle_given_rho(oracle, sc.params, x, v, y, u, g["rho"], fsample=fs, asample=as_, nbr_mode=nbr_mode)
        rep = {}
        compare_step(g, ref, sc.params, x, y, fs=fs, as_=as_, report=rep, ref_rho=refc)
        for kk, vv in rep.items():
            worst[kk] = max(worst.get(kk, 0.0), vv)
        x, v, y, u = g["x1"], g["v1"], g["y1"], g["u1"]
    print("[parity] worst errors:", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    sim.close()
    return worst


def test_config0_ten_steps():
    worst = chained_parity(scenes.config0(), 10)
    assert worst["rho"] < 1e-4


def test_config0c_coupling_active():
    sc = scenes.config0c()
    sim = sph.create(sc, flags=sph.FLAG_DIAGNOSTICS)
    sim.step(1)
    assert sim.read(sph.TOUCHED).sum() > 0
    assert (sim.read(sph.AGENT_COUNTS)[:, 3] > 0).all()
    sim.close()
    chained_parity(sc, 4)


def test_small_ragged_scene():
    chained_parity(scenes.small_dam(nx=13, ny=7, nz=11, n_agents=37, agents="inside"), 3)


def test_agents_above_and_upper():
    chained_parity(scenes.small_dam(nx=9, ny=9, nz=9, n_agents=50, agents="upper"), 2)


def test_dense_clump_against_oracle():
    """Cells with ~200 particles: neighbour counts in the hundreds, halo rows
    staged in several LDS windows, rows whose candidates overflow a mask."""
    sc = scenes.clumped_dam()
    worst = chained_parity(sc, 2)
    assert worst["rho"] < 1e-4


def test_wide_coupling_radius():
    """r_couple = 4h: the coupling stencil has 9 x 9 = 81 fluid rows, more than a
    wavefront's 64 lanes, so the agents' flattened gather takes two row groups."""
    sc = scenes.small_dam(nx=12, ny=10, nz=12, n_agents=30, agents="inside")
    sc.params["r_couple"] = float(np.float32(4 * sc.params["h"]))
    worst = chained_parity(sc, 2)
    print(f"[parity] wide coupling worst {worst}", flush=True)


def test_paper_literal_kernel_constants():
    sc = scenes.small_dam(nx=10, ny=8, nz=10, n_agents=12)
    sc.params["kernel_norm"] = 1
    chained_parity(sc, 2)


def test_config1_full_size_sampled_graph():
    """1,048,576 particles in the captured-graph launch path; float outputs on a sample."""
    sc = scenes.config1()
    print("[parity] config1 full size", flush=True)
    sim = sph.create(sc, flags=sph.FLAG_DIAGNOSTICS)
    sim.capture(1)
    sim.step(1)  # replays the graph
    x, v, y, u = state(sim)
    sim.step(1)
    g = gpu_fields(sim)
    rng = np.random.default_rng(11)
    fs = np.unique(np.concatenate([rng.choice(sc.n, 1500, replace=False), np.arange(64),
                                   np.arange(sc.n - 64, sc.n)]))
    as_ = np.arange(sc.n_agents)
    ref = oracle.step(sc.params, x, v, y, u, fsample=fs, asample=as_, nbr_mode=1)
    refc = oracle_given_rho(oracle, sc.params, x, v, y, u, g["rho"], fsample=fs, asample=as_, nbr_mode=1)
    rep = {}
    compare_step(g, ref, sc.params, x, y, fs=fs, as_=as_, report=rep, ref_rho=refc)
    print("[parity] config1 errors:", {k: f"{v:.2e}" for k, v in rep.items()}, flush=True)
    pairs = sim.read(sph.PAIR_COUNT)[0]
    assert pairs > 25 * sc.n * 2  # two steps with ~30 neighbours each
    sim.close()


def test_config2_full_size_sampled():
    """16,777,216 particles in two blocks of unequal height on a 2^24-cell grid,
    65,536 agents in flocks: integer outputs on every element, floats on a sample."""
    sc = scenes.config2()
    print("[parity] config2 full size", flush=True)
    sim = sph.create(sc, flags=sph.FLAG_DIAGNOSTICS)
    sim.step(1)
    x, v, y, u = state(sim)
    sim.step(1)
    g = gpu_fields(sim)
    rng = np.random.default_rng(12)
    fs = np.unique(np.concatenate([rng.choice(sc.n, 1000, replace=False), np.arange(32),
                                   np.arange(sc.n - 32, sc.n)]))
    as_ = np.unique(rng.choice(sc.n_agents, 256, replace=False))
    ref = oracle.step(sc.params, x, v, y, u, fsample=fs, asample=as_, nbr_mode=1)
    refc = oracle_given_rho(oracle, sc.params, x, v, y, u, g["rho"], fsample=fs, asample=as_, nbr_mode=1)
    rep = {}
    compare_step(g, ref, sc.params, x, y, fs=fs, as_=as_, report=rep, ref_rho=refc)
    print("[parity] config2 errors:", {k: f"{v:.2e}" for k, v in rep.items()}, flush=True)
    sim.close()


def test_graph_replay_equals_eager():
    sc = scenes.config0c()
    a = sph.create(sc)
    b = sph.create(sc)
    b.capture(3)
    for rep in range(3):
        a.step(3)
        b.step(3)  # graph replay
        for fa, fb in zip(state(a), state(b)):
            np.testing.assert_array_equal(fa, fb)
        a.step(1)  # eager work between replays
        b.step(1)
    a.close()
    b.close()


def test_profiled_steps_equal_plain_steps():
    """sph_step_profiled and sph_step_timed (events read back every 25 steps)
    advance the state exactly like sph_step."""
    sc = scenes.config0c()
    a = sph.create(sc)
    b = sph.create(sc)
    c = sph.create(sc)
    for n in (27, 3, 75):  # a chunk and a remainder, a remainder only, three chunks
        a.step(n)
        ph = b.step_profiled(n)
        assert set(ph) == {sph.phase_name(p) for p in range(sph.STEP_PHASES)}
        assert all(v > 0 for v in ph.values())
        kt = c.step_timed(n)
        assert set(kt) == {"density", "force_integrate"} and all(v > 0 for v in kt.values())
        for fa, fb, fc in zip(state(a), state(b), state(c)):
            np.testing.assert_array_equal(fa, fb)
            np.testing.assert_array_equal(fa, fc)
    assert a.info()["steps"] == b.info()["steps"] == c.info()["steps"] == 105
    a.close()
    b.close()
    c.close()


def test_checkpoint_resume_is_bit_identical():
    sc = scenes.config0c()
    a = sph.create(sc)
    a.step(6)
    b = sph.create(sc)
    b.step(3)
    x, v, y, u = state(b)
    b.close()
    c = sph.Simulation(sc.params, x, v, y, u)
    c.step(3)
    for fa, fc in zip(state(a), state(c)):
        np.testing.assert_array_equal(fa, fc)
    a.close()
    c.close()


def test_batched_equals_plain_per_scene():
    specs = scenes.batched_specs(5, n_range=(300, 3000), a_range=(2, 20))
    scs = [scenes.batched_scene(sp, k) for k, sp in enumerate(specs)]
    bat = sph.create_batch(scs)
    bat.step(3)
    X, V, Y, U = state(bat)
    for s, sc in enumerate(scs):
        p = sph.create(sc)
        p.step(3)
        x, v, y, u = state(p)
        p0, p1 = bat.part_off[s], bat.part_off[s + 1]
        a0, a1 = bat.agent_off[s], bat.agent_off[s + 1]
        np.testing.assert_array_equal(X[p0:p1], x)
        np.testing.assert_array_equal(V[p0:p1], v)
        np.testing.assert_array_equal(Y[a0:a1], y)
        np.testing.assert_array_equal(U[a0:a1], u)
        p.close()
    bat.close()


def test_batched_parity_against_oracle():
    specs = scenes.batched_specs(3, n_range=(500, 2500), a_range=(3, 30))
    scs = [scenes.batched_scene(sp, k) for k, sp in enumerate(specs)]
    for sc in scs:  # put the agents inside the fluid so coupling is exercised
        lo, hi = sc.x.min(0), sc.x.max(0)
        sc.y[:] = (lo + (hi - lo) * np.linspace(0.2, 0.8, len(sc.y))[:, None]).astype(np.float32)
    bat = sph.create_batch(scs, flags=sph.FLAG_DIAGNOSTICS)
    bat.step(1)
    g_all = gpu_fields(bat)
    for s, sc in enumerate(scs):
        p0, p1 = bat.part_off[s], bat.part_off[s + 1]
        a0, a1 = bat.agent_off[s], bat.agent_off[s + 1]
        ref = oracle.step(sc.params, sc.x, sc.v, sc.y, sc.u)
        refc = oracle_given_rho(oracle, sc.params, sc.x, sc.v, sc.y, sc.u, g_all["rho"][p0:p1])
        nc = len(ref["off"])
        c0 = sum(oracle.grid(scs[t].params)[3] + 1 for t in range(s))
        ac0 = sum(oracle.grid(scs[t].params, True)[3] + 1 for t in range(s))
        g = {}
        for k, val in g_all.items():
            if k in ("off",):
                g[k] = val[c0:c0 + nc]
            elif k == "aoff":
                g[k] = val[ac0:ac0 + len(ref["aoff"])]
            elif k in ("akey", "asorted", "y1", "u1", "force", "steer", "acounts"):
                g[k] = val[a0:a1]
            else:
                g[k] = val[p0:p1]
        compare_step(g, ref, sc.params, sc.x, sc.y, ref_rho=refc)
    bat.close()


def test_edge_inputs():
    # no agents
    sc = scenes.small_dam(nx=6, ny=5, nz=7, n_agents=0)
    chained_parity(sc, 1)
    # particles on the max wall, on the min corner, coincident pairs, and a lone particle
    sc = scenes.small_dam(nx=6, ny=5, nz=7, n_agents=3)
    bmax = np.asarray(sc.params["box_max"], np.float32)
    extra = np.array([bmax, [0, 0, 0], [0.3, 0.3, 0.3], [0.3, 0.3, 0.3], [0.9, 0.7, 0.9]], np.float32)
    sc.x = np.concatenate([sc.x, extra])
    sc.v = np.concatenate([sc.v, np.zeros_like(extra)])
    chained_parity(sc, 2)


def test_single_particle_and_no_fluid():
    p = scenes.default_params(0.05, 5e-4, (0, 0, 0), (1, 1, 1))
    x = np.array([[0.5, 0.5, 0.9]], np.float32)
    v = np.array([[0.1, 0.0, 0.2]], np.float32)
    sim = sph.Simulation(p, x, v, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32))
    sim.step(1)
    ref = oracle.step(p, x, v, np.zeros((0, 3)), np.zeros((0, 3)))
    np.testing.assert_allclose(sim.read(sph.POS), ref["x1"], rtol=1e-6)
    sim.close()
    y = np.array([[0.5, 0.5, 0.5], [0.55, 0.5, 0.5]], np.float32)
    u = np.array([[0.5, 0, 0], [0, 0.5, 0]], np.float32)
    sim = sph.Simulation(p, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), y, u,
                         flags=sph.FLAG_DIAGNOSTICS)
    sim.step(1)
    ref = oracle.step(p, np.zeros((0, 3)), np.zeros((0, 3)), y, u)
    np.testing.assert_allclose(sim.read(sph.AGENT_STEER), ref["steer"], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(sim.read(sph.AGENT_POS), ref["y1"], rtol=1e-6)
    sim.close()


def test_nonfinite_state_is_reported():
    sc = scenes.small_dam(nx=5, ny=5, nz=5, n_agents=2)
    sc.v[3, 1] = np.nan
    sim = sph.create(sc, flags=sph.FLAG_CHECK_FINITE)
    with pytest.raises(sph.SphError) as ei:
        sim.step(1)
    assert ei.value.status == sph.ENONFINITE
    sim.close()


def test_diagnostics_need_the_flag():
    sc = scenes.small_dam(nx=5, ny=5, nz=5, n_agents=2)
    sim = sph.create(sc)
    sim.step(1)
    with pytest.raises(sph.SphError) as ei:
        sim.read(sph.ACC_INT)
    assert ei.value.status == sph.ESTATE
    sim.close()


def test_walls_per_element():
    """Every particle and agent is compared, position and velocity, against
    the oracle in a step that carries them through the walls: both sides must
    take the same reflection decisions, and the displacement of each element
    must agree to 1e-4 of the displacement scale (plus float32 rounding)."""
    p, x, v, y, u, dt = scenes.wall_scene()
    sim = sph.Simulation(p, x, v, y, u, flags=sph.FLAG_DIAGNOSTICS)
    for k in range(2):
        print(f"[parity] walls step {k}", flush=True)
        sim.step(1)
        g = gpu_fields(sim)
        ref = oracle.step(p, x, v, y, u)
        refc = oracle_given_rho(oracle, p, x, v, y, u, g["rho"])
        rep = {}
        compare_step(g, ref, p, x, y, report=rep, ref_rho=refc)
        print("[parity] walls:", rep, flush=True)
        assert rep["x_wall_ambiguous"] == 0 and rep["y_wall_ambiguous"] == 0
        if k == 0:
            # 6 single walls, 5 corners (2 or 3 walls), 2 edges and the particle on a wall
            assert rep["x_wall_reflections"] == 6 + (3 + 3 + 3 + 3 + 3) + 4 + 1
            assert rep["y_wall_reflections"] == 1 + 1 + 1 + 3
            # every reflected coordinate is inside the box, mirrored by its overshoot
            gx = g["x1"].astype(np.float64)
            assert (gx >= 0).all() and (gx <= 1).all()
        x, v, y, u = g["x1"], g["v1"], g["y1"], g["u1"]
    sim.close()
