"""The parity comparison itself, on the CPU: it must accept the oracle's own
step rounded to float32 and reject plausible mistakes in the position update
and the walls.  The mistakes are planted in a copy of the oracle's output."""
import numpy as np
import pytest

import oracle
from paper_2311_15088_amd import scenes

from parity import compare_step


def _as_gpu(ref):
    g = {}
    for k in ("key", "off", "sorted", "akey", "aoff", "asorted", "nbr", "touched"):
        g[k] = ref[k].copy()
    for k in ("rho", "a_int", "a_coup", "force", "steer", "x1", "v1", "y1", "u1"):
        g[k] = ref[k].astype(np.float32)
    g["acounts"] = np.stack([ref[k] for k in ("n_sep", "n_ali", "n_coh", "n_cpl")], 1)
    return g


@pytest.fixture(scope="module")
def moving_state():
    """config 0c after one oracle step: fluid and agents in motion."""
    sc = scenes.config0c()
    r = oracle.step(sc.params, sc.x, sc.v, sc.y, sc.u)
    x, v = r["x1"].astype(np.float32), r["v1"].astype(np.float32)
    y, u = r["y1"].astype(np.float32), r["u1"].astype(np.float32)
    return sc.params, x, v, y, u, oracle.step(sc.params, x, v, y, u)


def test_oracle_rounded_to_float32_passes(moving_state):
    p, x, v, y, u, ref = moving_state
    rep = {}
    compare_step(_as_gpu(ref), ref, p, x, y, report=rep)
    assert rep["x_disp"] < 1e-6 and rep["y_disp"] < 1e-6


@pytest.mark.parametrize("mistake", ["no_position_update", "explicit_euler", "half_dt", "no_gravity_in_x"])
def test_position_update_mistakes_are_caught(moving_state, mistake):
    p, x, v, y, u, ref = moving_state
    g = _as_gpu(ref)
    dt = float(np.float32(p["dt"]))
    x64 = x.astype(np.float64)
    if mistake == "no_position_update":
        g["x1"] = x.copy()
    elif mistake == "explicit_euler":  # x' from the old velocity
        g["x1"] = (x64 + dt * v.astype(np.float64)).astype(np.float32)
    elif mistake == "half_dt":
        g["x1"] = (x64 + 0.5 * (ref["x1"] - x64)).astype(np.float32)
    else:  # x' moved with the velocity before gravity was added
        vg = ref["v1"] - dt * np.asarray(p["gravity"], np.float64)
        g["x1"] = (x64 + dt * vg).astype(np.float32)
    with pytest.raises(AssertionError):
        compare_step(g, ref, p, x, y)


@pytest.mark.parametrize("mistake", ["no_reflection", "no_restitution", "no_clamp_mirror", "agents_unreflected"])
def test_wall_mistakes_are_caught(mistake):
    p, x, v, y, u, _ = scenes.wall_scene()
    ref = oracle.step(p, x, v, y, u)
    g = _as_gpu(ref)
    rep = {}
    compare_step(g, ref, p, x, y, report=rep)  # the unaltered copy passes
    if mistake == "no_reflection":  # positions clamped, velocities kept
        g["x1"] = np.clip(ref["x1f"], 0.0, 1.0).astype(np.float32)
        g["v1"] = ref["v1f"].astype(np.float32)
    elif mistake == "no_restitution":  # mirrored but the velocity only flipped
        out = (ref["x1f"] < 0) | (ref["x1f"] > 1)
        g["v1"] = np.where(out, -ref["v1f"], ref["v1f"]).astype(np.float32)
    elif mistake == "no_clamp_mirror":  # clamped onto the wall instead of mirrored
        out = (ref["x1f"] < 0) | (ref["x1f"] > 1)
        g["x1"] = np.where(out, np.clip(ref["x1f"], 0, 1), ref["x1"]).astype(np.float32)
    else:
        g["y1"] = np.clip(ref["y1f"], 0.0, 1.0).astype(np.float32)
        g["u1"] = ref["u1f"].astype(np.float32)
    with pytest.raises(AssertionError):
        compare_step(g, ref, p, x, y)
