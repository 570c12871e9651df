"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (float32 GPU against float64 reference, same float32 start state):
  * integer / index outputs (cell keys, offsets, sorted ids, neighbour and
    agent counts): bit-exact;
  * density: per-element relative error <= 1e-4;
  * vector fields (accelerations, forces, steering, new velocity): every
    element within 1e-4 of the field's largest magnitude,
    max_i |g_i - c_i|_inf / max_i |c_i|_inf <= 1e-4.  Interior SPH forces are
    sums of O(1) pair terms that cancel to O(1e-3); float32 rounding of those
    terms (~1e-7 each) cannot keep a plain per-element relative bound there.
    The per-element figure with a floor of 1e-3 of the field scale ("_floor")
    is asserted as well, at 1e-4, for a_int, the agents' coupling force and
    the steering.
  * forces given the density: the oracle is run a second time with the GPU's
    own densities in its force terms (``oracle.step(..., rho_in=...)``), and
    a_int, a_coup and the agents' force must then agree per element (floor
    metric) to 1e-4: the force arithmetic itself, separated from the density
    it is fed.
  * the fluid's coupling acceleration per element: the agent sits at rest
    density, so its pressure term on particle i carries rho_i - rho0, and a
    density right to ~3e-7 (well inside its own 1e-4 bar) becomes a pressure
    term that is off by 3e-7 rho / |rho_i - rho0| -- 1e-3 and more where
    rho_i is within a few tenths of rho0.  Its floor metric is asserted
    against 1e-4 plus exactly that propagated part, which the two oracle runs
    give: floor_err(oracle with the GPU's densities, oracle).
  * new positions: the one-step displacement x' - x of every element is
    compared with the oracle's, within 1e-4 of the displacement field's
    largest magnitude plus the rounding of a float32 position (one unit in the
    last place of x': the rounding of x + dt v' and of a wall's mirror image);
    the per-element relative error of x' itself is reported beside it.
  * walls: every element is compared.  A reflection is a discrete decision
    taken on the unreflected position; where the oracle's unreflected
    coordinate lies within the comparison's own tolerance of a wall, the
    other side may decide the other way, and the element is then compared
    with whichever of the two outcomes (reflected or not, both built from the
    oracle's unreflected state) is nearer.  Elsewhere both sides must take
    the oracle's decision.
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


def ulp32(a):
    """Spacing of float32 numbers at |a| (as float64)."""
    return np.spacing(np.abs(np.asarray(a, np.float64)).astype(np.float32)).astype(np.float64)


def _state_errs(g_pos, g_vel, ref, key, p0, params, sel, prefix, errs, info):
    """Displacement and velocity of one set (fluid: key 'x', agents: key 'y')."""
    pos1, vel1 = ("x1", "v1") if key == "x" else ("y1", "u1")
    gx = np.asarray(g_pos, np.float64)[sel].reshape(-1, 3)
    gv = np.asarray(g_vel, np.float64)[sel].reshape(-1, 3)
    cx = np.asarray(ref[pos1], np.float64)[sel].reshape(-1, 3)
    cv = np.asarray(ref[vel1], np.float64)[sel].reshape(-1, 3)
    fx = np.asarray(ref[pos1 + "f"], np.float64)[sel].reshape(-1, 3)
    fv = np.asarray(ref[vel1 + "f"], np.float64)[sel].reshape(-1, 3)
    x0 = np.asarray(p0, np.float64)[sel].reshape(-1, 3)
    if len(cx) == 0:
        return
    lo = np.asarray(params["box_min"], np.float32).astype(np.float64)
    hi = np.asarray(params["box_max"], np.float32).astype(np.float64)
    e = float(np.float32(params["wall_restitution"]))
    sd = np.abs(cx - x0).max()  # displacement scale
    sv = np.abs(cv).max()       # velocity scale
    # allowance for the float32 rounding of a position, per element
    ux = np.maximum(ulp32(cx), ulp32(gx))
    # the other outcome of each wall decision, from the oracle's unreflected state
    out_lo, out_hi = fx < lo, fx > hi
    refl = out_lo | out_hi
    alt_x = np.where(refl, fx, np.where(fx - lo < hi - fx, 2.0 * lo - fx, 2.0 * hi - fx))
    alt_x = np.clip(alt_x, lo, hi)
    alt_v = np.where(refl, fv, -e * fv)
    # decisions within the tolerance of the comparison itself may go either way
    margin = TOL_REL * sd + 2.0 * np.maximum(ux, ulp32(np.maximum(np.abs(lo), np.abs(hi))))
    amb = (np.abs(fx - lo) <= margin) | (np.abs(fx - hi) <= margin)
    ex = np.abs(gx - cx)
    ev = np.abs(gv - cv)
    ex_alt = np.abs(gx - alt_x)
    ev_alt = np.abs(gv - alt_v)
    # per element: the nearer outcome where the decision is ambiguous (both
    # coordinates judged together so x' and v' come from one outcome)
    use_alt = amb & (np.maximum(ex_alt / (TOL_REL * sd + ux), ev_alt / max(sv, 1e-30)) <
                     np.maximum(ex / (TOL_REL * sd + ux), ev / max(sv, 1e-30)))
    ex = np.where(use_alt, ex_alt, ex)
    ev = np.where(use_alt, ev_alt, ev)
    errs[prefix + "disp"] = float((np.maximum(ex - ux, 0.0) / sd).max()) if sd > 0 else float(
        np.maximum(ex - ux, 0.0).max())
    errs[prefix + "vel"] = float(ev.max() / sv) if sv > 0 else float(ev.max())
    nz = np.abs(cx) > 0
    errs[prefix + "pos_elem"] = float((ex[nz] / np.abs(cx[nz])).max()) if nz.any() else 0.0
    info[prefix + "wall_reflections"] = int(refl.sum())
    info[prefix + "wall_ambiguous"] = int(amb.sum())
    info[prefix + "wall_other_outcome"] = int(use_alt.sum())


def compare_step(gpu: dict, ref: dict, params: dict, x0, y0, fs=None, as_=None, report=None, ref_rho=None):
    """Assert parity of one step.  ``gpu`` / ``ref`` map field names to arrays in id
    order; ``x0`` / ``y0`` are the float32 fluid and agent positions the step
    started from (id order); ``fs`` / ``as_`` restrict the float comparisons to
    sampled ids; ``ref_rho`` is the oracle's step with the GPU's densities in
    its force terms (``oracle_given_rho``)."""
    errs = {}
    info = {}
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
    bounds = {}
    for name in ("a_int", "a_coup"):
        if name in gpu:
            errs[name] = rel_scale_err(gpu[name][f], ref[name][f])
            errs[name + "_floor"] = floor_err(gpu[name][f], ref[name][f])
    for name in ("force", "steer"):
        if name in gpu and len(ref[name][a]):
            errs[name] = rel_scale_err(gpu[name][a], ref[name][a])
            errs[name + "_floor"] = floor_err(gpu[name][a], ref[name][a])
    if ref_rho is not None:
        for name, sel in (("a_int", f), ("a_coup", f), ("force", a)):
            if name in gpu and len(ref[name][sel]):
                errs[name + "_given_rho_floor"] = floor_err(gpu[name][sel], ref_rho[name][sel])
        if "a_coup" in gpu:
            info["a_coup_floor_from_density"] = floor_err(ref_rho["a_coup"][f], ref["a_coup"][f])
            bounds["a_coup_floor"] = TOL_REL + info["a_coup_floor_from_density"]
    elif "a_coup" in gpu:
        bounds["a_coup_floor"] = float("inf")  # only with the density-conditioned run
    # --- new state, every element ---
    _state_errs(gpu["x1"], gpu["v1"], ref, "x", x0, params, f, "x_", errs, info)
    if len(ref["y1"][a]):
        _state_errs(gpu["y1"], gpu["u1"], ref, "y", y0, params, a, "y_", errs, info)
    errs["x1"] = rel_scale_err(gpu["x1"][f], ref["x1"][f])
    if report is not None:
        report.update(errs)
        report.update({"bound_" + k: v for k, v in bounds.items() if np.isfinite(v)})
        report.update(info)
    bad = {k: v for k, v in errs.items() if not (v <= bounds.get(k, TOL_REL))}
    assert not bad, f"parity errors above the bar: {bad} (bounds {bounds}; all: {errs}; {info})"
    return errs


def oracle_given_rho(oracle, params, x, v, y, u, gpu_rho, **kw):
    """The oracle's step with the GPU's densities (id order) in its force terms."""
    return oracle.step(params, x, v, y, u, rho_in=np.asarray(gpu_rho, np.float64), **kw)
