"""Voxel density at cube corners -- the reference for the library's voxel pass.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy in float64;
candidate particles come from scipy's k-d tree (a library search that only
narrows the candidates; membership is decided below).

"Voxel Density" section: at a cube corner x,
    phi(x) = |x - xbar| - rbar,   xbar = sum_i w_i x_i,   rbar = sum_i w_i r_i,
    w_i = k(|x - x_i| / R) / sum_j k(|x - x_j| / R),   k(s) = (1 - s^2)^3,
over the particles within the neighbourhood radius R of x.

Readings of this project (the paper leaves them open):
  * corners are x_c = box_min + c * spacing for c = 0 .. floor((box_max -
    box_min) / spacing) on each axis, x fastest, each coordinate rounded to
    float32 as fl(box_min + fl(c * spacing));
  * i is in the neighbourhood of x when the float32 squared distance (the
    oracle's predicate: per-axis differences, then fl(dz^2 + fl(dy^2 +
    fl(dx^2))) with the two outer steps fused) is below fl32(R * R); that
    integer decision is taken in the same precision on both sides;
  * every particle has the same radius r, so rbar = r whenever the
    neighbourhood is not empty; a corner with an empty neighbourhood has
    phi = +inf (outside any surface).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from . import fp32


def corner_dims(p: Dict, spacing: float) -> Tuple[int, int, int]:
    lo = np.asarray(p["box_min"], np.float64)
    hi = np.asarray(p["box_max"], np.float64)
    gs = float(np.float32(spacing))
    return tuple(int(np.floor((hi[k] - lo[k]) / gs)) + 1 for k in range(3))


def corners(p: Dict, spacing: float) -> np.ndarray:
    """[nz * ny * nx, 3] float32 corner positions, x fastest."""
    dims = corner_dims(p, spacing)
    gs = np.float32(spacing)
    lo = np.asarray(p["box_min"], np.float32)
    ax = [lo[k] + np.arange(dims[k], dtype=np.float32) * gs for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float32)


def inside_f32(q: np.ndarray, x: np.ndarray, r2: np.float32) -> np.ndarray:
    """float32 predicate |x - q|^2 < r2 for one corner q against points x
    (the oracle's squared distance, ``oracle/fp32.py``)."""
    d = x - q[None, :]
    return fp32.dist2(d[:, 0], d[:, 1], d[:, 2]) < r2


def field(p: Dict, x, spacing: float, radius: float, particle_radius: float, sample=None) -> np.ndarray:
    """phi at every corner (float64, x fastest); +inf where no particle is within R.
    sample: corner indices to evaluate (the others are NaN)."""
    from scipy.spatial import cKDTree

    x = np.ascontiguousarray(np.asarray(x, np.float32)).reshape(-1, 3)
    q = corners(p, spacing)
    R = float(np.float32(radius))
    r2 = np.float32(R * R)
    r = float(np.float32(particle_radius))
    which = np.arange(q.shape[0]) if sample is None else np.asarray(sample, np.int64)
    out = np.full(q.shape[0], np.inf if sample is None else np.nan)
    out[which] = np.inf
    if x.shape[0] == 0:
        return out
    tree = cKDTree(x.astype(np.float64))
    cand = tree.query_ball_point(q[which].astype(np.float64), R * (1.0 + 1e-5))
    for c, idx in zip(which, cand):
        if not idx:
            continue
        idx = np.asarray(idx)
        idx = idx[inside_f32(q[c], x[idx], r2)]
        if idx.size == 0:
            continue
        xi = x[idx].astype(np.float64)
        xc = q[c].astype(np.float64)
        s = np.linalg.norm(xc[None, :] - xi, axis=1) / R
        k = np.maximum(1.0 - s * s, 0.0) ** 3
        tot = k.sum()
        if tot <= 0.0:
            continue
        w = k / tot
        xbar = (w[:, None] * xi).sum(axis=0)
        rbar = w.sum() * r
        out[c] = np.linalg.norm(xc - xbar) - rbar
    return out
