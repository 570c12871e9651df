"""Execution forms of the step (per-phase launches, one fused persistent launch,
kernel variants, tile widths, graphs, batched scenes) give bit-identical
results, and the autotuner leaves the simulation state untouched."""
import numpy as np
import pytest

import paper_2311_15088_amd as sph
from paper_2311_15088_amd import scenes

pytestmark = pytest.mark.gpu


def state(sim):
    return [sim.read(f) for f in (sph.POS, sph.VEL, sph.AGENT_POS, sph.AGENT_VEL, sph.DENSITY, sph.NBR_COUNT)]


def same(a, b):
    for fa, fb in zip(a, b):
        np.testing.assert_array_equal(fa, fb)


WIDTHS = (32, 1, 7, 16, 8)


def run(sc, steps, fused=0, variant=0, tile_x=32, graph=False, batch=None):
    sim = sph.create_batch(batch) if batch is not None else sph.create(sc)
    sim.set_tuning(fused, variant, tile_x)
    if graph:
        sim.capture(steps)
    sim.step(steps)
    out = state(sim)
    sim.close()
    return out


def test_variants_and_tile_widths_are_bit_identical():
    sc = scenes.small_dam(nx=20, ny=9, nz=15, n_agents=30, agents="inside")
    print(f"[forms] n={sc.n}", flush=True)
    ref = run(sc, 4)
    for v in range(sph.variant_count(0)):
        for tx in WIDTHS + ((64, 48) if sph.variant_tile_max(0, v) >= 64 else ()):
            same(ref, run(sc, 4, 0, v, tx))


def test_dense_clump_takes_every_path_bit_identically():
    """A clump of ~200 particles per cell: halo rows longer than every LDS
    window (staged in pieces) and rows with more candidates than a 64-bit mask
    records (retested in the force pass).  Every variant and width must agree
    bit for bit."""
    sc = scenes.clumped_dam()
    print(f"[forms] clump n={sc.n}", flush=True)
    ref = run(sc, 2)
    for v in range(sph.variant_count(0)):
        for tx in (32, 1, 5) + ((64,) if sph.variant_tile_max(0, v) >= 64 else ()):
            print(f"[forms] clump variant {v} tile_x {tx}", flush=True)
            same(ref, run(sc, 2, 0, v, tx))
    for v in range(sph.variant_count(1)):
        same(ref, run(sc, 2, 1, v, 32))


def test_fused_step_matches_per_phase_launches():
    sc = scenes.config0c()
    ref = run(sc, 6)
    for v in range(sph.variant_count(1)):
        for tx in (32, 8, 13):
            print(f"[forms] fused variant {v} tile_x {tx}", flush=True)
            same(ref, run(sc, 6, 1, v, tx))
    same(ref, run(sc, 6, 1, 0, 32, graph=True))


def test_fused_batched_matches_plain_per_scene():
    specs = scenes.batched_specs(6, n_range=(300, 4000), a_range=(2, 40))
    scs = [scenes.batched_scene(sp, k) for k, sp in enumerate(specs)]
    bat = sph.create_batch(scs)
    bat.set_tuning(1, 0, 32)
    bat.capture(3)
    bat.step(3)
    X, V, Y, U = (bat.read(f) for f in (sph.POS, sph.VEL, sph.AGENT_POS, sph.AGENT_VEL))
    for s, sc in enumerate(scs):
        x, v, y, u, _, _ = run(sc, 3)
        p0, p1 = bat.part_off[s], bat.part_off[s + 1]
        a0, a1 = bat.agent_off[s], bat.agent_off[s + 1]
        np.testing.assert_array_equal(X[p0:p1], x)
        np.testing.assert_array_equal(V[p0:p1], v)
        np.testing.assert_array_equal(Y[a0:a1], y)
        np.testing.assert_array_equal(U[a0:a1], u)
    bat.close()


def test_two_row_tiles_batched_equal_plain_per_scene():
    """Two-row tiles over batched scenes of different grids (odd and even
    row counts along y, so some tiles hold one row): each scene's result is
    the plain one-scene step's, bit for bit."""
    specs = scenes.batched_specs(5, n_range=(300, 4000), a_range=(2, 40))
    scs = [scenes.batched_scene(sp, k) for k, sp in enumerate(specs)]
    two_row = [v for v in range(sph.variant_count(0)) if "ty2" in (sph.variant_name(0, v) or "")]
    assert two_row
    plain = [run(sc, 3) for sc in scs]
    for v in two_row:
        print(f"[forms] batched two-row variant {v}", flush=True)
        bat = sph.create_batch(scs)
        bat.set_tuning(0, v, 16)
        bat.step(3)
        X, V, Y, U = (bat.read(f) for f in (sph.POS, sph.VEL, sph.AGENT_POS, sph.AGENT_VEL))
        for s in range(len(scs)):
            x, vv, y, u, _, _ = plain[s]
            p0, p1 = bat.part_off[s], bat.part_off[s + 1]
            a0, a1 = bat.agent_off[s], bat.agent_off[s + 1]
            np.testing.assert_array_equal(X[p0:p1], x)
            np.testing.assert_array_equal(V[p0:p1], vv)
            np.testing.assert_array_equal(Y[a0:a1], y)
            np.testing.assert_array_equal(U[a0:a1], u)
        bat.close()


def test_closure_attached_to_a_fused_context_steps_per_phase():
    """Attaching a closure turns a fused context back to per-phase launches
    with its kernel variant's tiles (here a two-row variant); with a bound of
    0 the controller always takes the exact gather, so the steps equal plain
    ones."""
    sc = scenes.config0c()
    v2 = [v for v in range(sph.variant_count(0)) if "ty2" in (sph.variant_name(0, v) or "")][0]
    a = sph.create(sc)
    a.set_tuning(0, v2, 16)
    a.set_tuning(1, 0, 16)  # fused; the per-phase variant stays the two-row one
    a.step(1)
    cl = sph.Closure(scenes.mlp_flat(scenes.mlp_init()))
    a.attach_closure(cl, check_every=2, max_rel_rms=0.0)
    assert a.tuning()["fused"] == 0
    a.step(3)
    b = sph.create(sc)
    b.step(4)
    same(state(b), state(a))
    a.attach_closure(None)
    a.close()
    b.close()
    cl.close()


def test_autotune_keeps_state_and_picks_a_valid_form():
    sc = scenes.small_dam(nx=24, ny=10, nz=20, n_agents=40, agents="inside")
    a = sph.create(sc)
    a.step(2)
    before = state(a)
    best = a.autotune(2)
    print("[forms] autotune picked", best, flush=True)
    assert best["ms_per_step"] > 0 and best["name"]
    same(before, state(a))  # tuning did not advance the simulation
    assert a.tuning()["fused"] == best["fused"] and a.tuning()["tile_x"] == best["tile_x"]
    a.step(3)
    b = sph.create(sc)
    b.step(5)
    same(state(a), state(b))
    a.close()
    b.close()


def test_invalid_tuning_is_rejected():
    sc = scenes.small_dam(nx=5, ny=5, nz=5, n_agents=2)
    sim = sph.create(sc)
    wide = [v for v in range(sph.variant_count(0)) if sph.variant_tile_max(0, v) == 64]
    narrow = [v for v in range(sph.variant_count(0)) if sph.variant_tile_max(0, v) == 32]
    assert wide and narrow and sph.variant_tile_max(1, 0) == 32
    sim.set_tuning(0, wide[0], 64)
    for bad in ((2, 0, 16), (0, 99, 16), (0, 0, 0), (0, wide[0], 65), (0, narrow[0], 33), (1, 0, 33), (1, 99, 8)):
        with pytest.raises(sph.SphError) as ei:
            sim.set_tuning(*bad)
        assert ei.value.status == sph.EINVAL
    sim.close()


def test_fused_abort_is_reported_and_leaves_the_state():
    """The fused step's sticky abort flag (what a timed-out grid barrier
    raises), set from the host: the fused kernel leaves at entry, so nothing
    hangs and the state is untouched; sph_read and every later sph_step report
    SPH_EHIP; clearing the flag re-arms the fused step."""
    sc = scenes.config0c()
    sim = sph.create(sc)
    sim.set_tuning(1, 0, 32)
    sim.step(2)
    before = state(sim)
    sim.set_abort(True)
    try:
        sim.step(1)  # enqueued; the flag's host copy may not have landed yet
    except sph.SphError as e:
        assert e.status == sph.EHIP
    with pytest.raises(sph.SphError) as ei:
        sim.read(sph.POS)
    assert ei.value.status == sph.EHIP
    with pytest.raises(sph.SphError) as ei:
        sim.step(1)
    assert ei.value.status == sph.EHIP
    sim.set_abort(False)
    same(before, state(sim))  # the aborted launch wrote nothing
    sim.step(1)
    ref = sph.create(sc)
    ref.step(3)
    same(state(ref), state(sim))
    ref.close()
    sim.close()


def test_abort_flag_does_not_touch_per_phase_steps():
    sc = scenes.config0c()
    sim = sph.create(sc)
    sim.step(1)  # per-phase launches never read the flag
    sim.set_abort(False)
    sim.step(1)
    ref = sph.create(sc)
    ref.step(2)
    same(state(ref), state(sim))
    ref.close()
    sim.close()


def test_default_form_is_the_documented_one_and_equals_variant_zero():
    """A context starts in the per-phase form with variant 1 (256-thread
    blocks in both fluid passes) and 32-cell tiles, and steps bit-identically
    to the 512-thread density form (variant 0)."""
    sc = scenes.config0c()
    sim = sph.create(sc)
    t = sim.tuning()
    assert (t["fused"], t["variant"], t["tile_x"]) == (0, 1, 32)
    assert sph.variant_name(0, t["variant"]) == "bd256_win512_512"
    sim.step(3)
    got = state(sim)
    sim.close()
    same(got, run(sc, 3, fused=0, variant=0, tile_x=32))
