"""Obstacle Grid and obstacle avoidance (sph_obstacles_set) against the
oracle: the avoidance acceleration from oracle/obstacles.py is given to the
oracle's step as a further steering term, and every field of the step is
compared as in the plain parity tests."""
import numpy as np
import pytest

import oracle
import paper_2311_15088_amd as sph
from oracle import obstacles
from paper_2311_15088_amd import scenes
from parity import compare_step, oracle_given_rho
from test_gpu_parity import gpu_fields, state

pytestmark = pytest.mark.gpu


def _scene_and_boxes():
    sc = scenes.small_dam(nx=16, ny=12, nz=16, n_agents=61, agents="inside")
    lo, hi = sc.x.min(0), sc.x.max(0)
    ext = hi - lo
    boxes = np.array([np.concatenate([lo + 0.30 * ext, lo + 0.55 * ext]),
                      np.concatenate([lo + 0.70 * ext, lo + 0.95 * ext])], np.float32)
    return sc, boxes


def test_obstacle_parity_against_oracle():
    sc, boxes = _scene_and_boxes()
    spacing, weight = 0.02, 0.8
    sim = sph.create(sc, flags=sph.FLAG_DIAGNOSTICS)
    sim.set_obstacles(boxes, spacing, weight)
    x, v, y, u = sc.x, sc.v, sc.y, sc.u
    touched = 0
    for k in range(3):
        acc = obstacles.avoidance(sc.params, y, boxes, spacing, weight)
        touched = max(touched, int((np.abs(acc).sum(1) > 0).sum()))
        print(f"[obstacles] step {k}: {int((np.abs(acc).sum(1) > 0).sum())} of {len(y)} agents steered", flush=True)
        sim.step(1)
        g = gpu_fields(sim)
        ref = oracle.step(sc.params, x, v, y, u, agent_acc=acc)
        refc = oracle_given_rho(oracle, sc.params, x, v, y, u, g["rho"], agent_acc=acc)
        compare_step(g, ref, sc.params, x, y, ref_rho=refc)
        x, v, y, u = g["x1"], g["v1"], g["y1"], g["u1"]
    assert touched >= 10
    sim.close()


def test_zero_weight_and_removal_leave_the_step_unchanged():
    sc, boxes = _scene_and_boxes()
    ref = sph.create(sc)
    ref.step(3)
    a = sph.create(sc)
    a.set_obstacles(boxes, 0.02, 0.0)  # weight 0: adds exactly 0 to every steering
    a.step(3)
    b = sph.create(sc)
    b.set_obstacles(boxes, 0.02, 0.8)
    b.set_obstacles([], 0.02, 0.8)     # removed again
    b.step(3)
    for s in (a, b):
        for got, want in zip(state(s), state(ref)):
            np.testing.assert_array_equal(got, want)
    c = sph.create(sc)
    c.set_obstacles(boxes, 0.02, 0.8)
    c.step(3)
    assert not np.array_equal(state(c)[3], state(ref)[3])  # the agents' velocities do change
    for s in (ref, a, b, c):
        s.close()


def test_obstacle_errors():
    sc, boxes = _scene_and_boxes()
    sim = sph.create(sc)
    bad = boxes.copy()
    bad[0, 3] = bad[0, 0] - 0.1  # max < min
    for args, code in (((bad, 0.02, 1.0), sph.EINVAL), ((boxes, 0.0, 1.0), sph.EINVAL),
                       ((boxes, 0.02, float("nan")), sph.EINVAL), ((boxes, 1e-6, 1.0), sph.ECAPACITY)):
        with pytest.raises(sph.SphError) as e:
            sim.set_obstacles(*args)
        assert e.value.status == code
    sim.close()
    specs = scenes.batched_specs(2, n_range=(300, 600), a_range=(2, 4))
    bat = sph.create_batch([scenes.batched_scene(sp, k) for k, sp in enumerate(specs)])
    with pytest.raises(sph.SphError) as e:
        bat.set_obstacles(boxes, 0.02, 1.0)
    assert e.value.status == sph.ENOTIMPL
    bat.close()
