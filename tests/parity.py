"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (float32 GPU against float64 reference, same float32 start state):
  * integer / index outputs (cell keys, offsets, sorted ids, neighbour and
    agent counts): bit-exact;
  * density: per-element relative error <= 1e-4;
  * vector fields (accelerations, forces, steering, new position / velocity):
    max_i |g_i - c_i|_inf / max_i |c_i|_inf <= 1e-4, i.e. relative to the
    field's own scale.  Interior SPH forces are sums of O(1) pair terms that
    cancel to O(1e-3); float32 rounding of those terms (~1e-7 each) cannot
    keep a per-element relative bound there, so the bound is taken against
    the field's largest magnitude.  The stricter per-element figure with a
    floor of 1e-3 of the field scale is reported alongside.
  * wall reflection is a discrete decision taken on values that differ in the
    last float32 bit between the two sides: a particle that one side reflects
    and the other does not must lie within rounding of the wall, and is then
    excluded from the velocity comparison.
"""
from __future__ import annotations

import numpy as np

TOL_REL = 1e-4


def rel_scale_err(g, c, mask=None):
    g = np.asarray(g, np.float64).reshape(len(g), -1)
    c = np.asarray(c, np.float64).reshape(len(c), -1)
    if mask is not None:
        g, c = g[mask], c[mask]
    if len(c) == 0:
        return 0.0
    scale = np.abs(c).max()
    if scale == 0.0:
        return float(np.abs(g).max())
    return float(np.abs(g - c).max() / scale)


def floor_err(g, c, floor=1e-3, mask=None):
    g = np.asarray(g, np.float64).reshape(len(g), -1)
    c = np.asarray(c, np.float64).reshape(len(c), -1)
    if mask is not None:
        g, c = g[mask], c[mask]
    if len(c) == 0:
        return 0.0
    cn = np.abs(c).max(1)
    den = np.maximum(cn, floor * cn.max())
    den[den == 0] = 1.0
    return float((np.abs(g - c).max(1) / den).max())


def elem_rel_err(g, c, mask=None):
    g = np.asarray(g, np.float64)
    c = np.asarray(c, np.float64)
    if mask is not None:
        g, c = g[mask], c[mask]
    if len(c) == 0:
        return 0.0
    return float((np.abs(g - c) / np.abs(c)).max())


def wall_mask(x_ref, box_min, box_max, tol=2e-6):
    """Particles whose reference position lies within ``tol`` (relative to the box) of a wall."""
    x = np.asarray(x_ref, np.float64)
    lo = np.asarray(box_min, np.float64)
    hi = np.asarray(box_max, np.float64)
    span = (hi - lo).max()
    return (np.abs(x - lo) < tol * span).any(1) | (np.abs(x - hi) < tol * span).any(1)


def compare_step(gpu: dict, ref: dict, params: dict, fs=None, as_=None, report=None):
    """Assert parity of one step.  ``gpu`` / ``ref`` map field names to arrays in id
    order; ``fs`` / ``as_`` restrict the float comparisons to sampled ids."""
    errs = {}
    # --- exact outputs ---
    np.testing.assert_array_equal(gpu["key"], ref["key"], err_msg="cell keys")
    np.testing.assert_array_equal(gpu["off"], ref["off"], err_msg="cell offsets")
    np.testing.assert_array_equal(gpu["sorted"], ref["sorted"], err_msg="sorted ids")
    np.testing.assert_array_equal(gpu["akey"], ref["akey"], err_msg="agent keys")
    np.testing.assert_array_equal(gpu["aoff"], ref["aoff"], err_msg="agent offsets")
    np.testing.assert_array_equal(gpu["asorted"], ref["asorted"], err_msg="agent sorted ids")
    f = slice(None) if fs is None else fs
    a = slice(None) if as_ is None else as_
    np.testing.assert_array_equal(gpu["nbr"][f], ref["nbr"][f], err_msg="neighbour counts")
    if "touched" in gpu:
        np.testing.assert_array_equal(gpu["touched"][f], ref["touched"][f], err_msg="agents touching a particle")
    if "acounts" in gpu:
        ac = gpu["acounts"][a]
        for k, name in enumerate(("n_sep", "n_ali", "n_coh", "n_cpl")):
            np.testing.assert_array_equal(ac[:, k], ref[name][a], err_msg=name)
    # --- float outputs ---
    errs["rho"] = elem_rel_err(gpu["rho"][f], ref["rho"][f])
    for name in ("a_int", "a_coup"):
        if name in gpu:
            errs[name] = rel_scale_err(gpu[name][f], ref[name][f])
            errs[name + "_floor"] = floor_err(gpu[name][f], ref[name][f])
    for name in ("force", "steer"):
        if name in gpu and len(ref[name][a]):
            errs[name] = rel_scale_err(gpu[name][a], ref[name][a])
            errs[name + "_floor"] = floor_err(gpu[name][a], ref[name][a])
    # new state: positions per-field scale; velocities excluding wall-rounding cases
    errs["x1"] = rel_scale_err(gpu["x1"][f], ref["x1"][f])
    near = wall_mask(ref["x1"][f], params["box_min"], params["box_max"])
    errs["v1"] = rel_scale_err(gpu["v1"][f], ref["v1"][f], mask=~near)
    if len(ref["y1"][a]):
        errs["y1"] = rel_scale_err(gpu["y1"][a], ref["y1"][a])
        near_a = wall_mask(ref["y1"][a], params["box_min"], params["box_max"])
        errs["u1"] = rel_scale_err(gpu["u1"][a], ref["u1"][a], mask=~near_a)
    if report is not None:
        report.update(errs)
    bad = {k: v for k, v in errs.items() if not k.endswith("_floor") and not (v <= TOL_REL)}
    assert not bad, f"parity errors above {TOL_REL}: {bad} (all: {errs})"
    return errs
