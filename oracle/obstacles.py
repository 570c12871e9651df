"""Obstacle Grid and obstacle avoidance -- the reference for the library's
obstacle term.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy.

Section "Underwater Agent Behaviors": the mesh normals of each obstacle are
attributed to the cells of an Obstacle Grid.  Section "Boid Motion and Agent
Fluid Interaction": a boid steers by the averaged normal vector of each
obstacle cell within its visual range, cells within its protection range
weighing more.

Readings of this project (the paper gives no formulas for these):
  * obstacles are axis-aligned boxes [lo, hi]; a box's mesh is its six faces,
    each sampled by a lattice of n_u + 1 by n_v + 1 vertices,
    n = max(1, ceil(extent / spacing)), at lo + ((hi - lo) i) / n in double,
    rounded to float32; every vertex carries its face's outward unit normal;
  * the Obstacle Grid is the agent grid (the Boid Grid); a vertex goes to the
    cell get_cell gives its float32 position (clamped like every key); a cell's
    normal is the mean of its vertices' normals;
  * a boid at y takes the 27 cells around its own cell; a cell holding
    vertices counts twice if its centre fl32(min + fl32((c + 1/2) d)) is
    within r_sep (the protection range) and once if within r_ali (the visual
    range), by float32 squared distances as for every membership decision;
    the avoidance acceleration is w_obs times the weighted sum of the cells'
    mean normals, added to the steering.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from . import fp32, grid


def mesh_vertices(boxes, spacing: float) -> Tuple[np.ndarray, np.ndarray]:
    """float32 vertex positions [m, 3] and their float64 outward normals [m, 3]."""
    boxes = np.asarray(boxes, np.float32).reshape(-1, 6)
    sp = float(np.float32(spacing))
    pts, nrm = [], []
    for b in boxes:
        lo, hi = b[:3].astype(np.float64), b[3:].astype(np.float64)
        for k in range(3):
            u, v = [a for a in range(3) if a != k]
            nu = max(1, int(np.ceil((hi[u] - lo[u]) / sp)))
            nv = max(1, int(np.ceil((hi[v] - lo[v]) / sp)))
            cu = lo[u] + ((hi[u] - lo[u]) * np.arange(nu + 1)) / nu
            cv = lo[v] + ((hi[v] - lo[v]) * np.arange(nv + 1)) / nv
            gv, gu = np.meshgrid(cv, cu, indexing="ij")
            for side, val in ((-1.0, lo[k]), (1.0, hi[k])):
                q = np.zeros((gu.size, 3))
                q[:, u] = gu.ravel()
                q[:, v] = gv.ravel()
                q[:, k] = val
                n = np.zeros((gu.size, 3))
                n[:, k] = side
                pts.append(q.astype(np.float32))
                nrm.append(n)
    if not pts:
        return np.zeros((0, 3), np.float32), np.zeros((0, 3))
    return np.concatenate(pts), np.concatenate(nrm)


def _agent_grid(p: Dict):
    dims, cell, inv, nc = grid(p, agent=True)
    return np.asarray(dims), np.float32(cell), np.float32(inv), nc, np.asarray(p["box_min"], np.float32)


def _cells(q: np.ndarray, mn, inv, dims) -> np.ndarray:
    """get_cell of float32 points: floor(fl32(fl32(q - min) * inv)), clamped."""
    t = (q.astype(np.float32) - mn) * inv
    f = np.floor(t)
    c = np.where(f >= 0, f, 0)
    return np.minimum(c, dims - 1).astype(np.int64)


def obstacle_grid(p: Dict, boxes, spacing: float) -> Tuple[np.ndarray, np.ndarray]:
    """Mean normal [cells, 3] (float64) and vertex count [cells] of every agent-grid cell."""
    dims, cell, inv, nc, mn = _agent_grid(p)
    pts, nrm = mesh_vertices(boxes, spacing)
    c = _cells(pts, mn, inv, dims)
    key = c[:, 0] + dims[0] * (c[:, 1] + dims[1] * c[:, 2])
    cnt = np.bincount(key, minlength=nc)
    tot = np.stack([np.bincount(key, weights=nrm[:, k], minlength=nc) for k in range(3)], axis=1)
    mean = np.zeros_like(tot)
    has = cnt > 0
    mean[has] = tot[has] / cnt[has, None]
    return mean, cnt


def avoidance(p: Dict, y, boxes, spacing: float, weight: float) -> np.ndarray:
    """w_obs * sum over the 27 cells around each agent of omega_c * mean normal_c, [na, 3] float64."""
    y = np.asarray(y, np.float32).reshape(-1, 3)
    dims, cell, inv, nc, mn = _agent_grid(p)
    mean, cnt = obstacle_grid(p, boxes, spacing)
    rs = float(np.float32(p["r_sep"]))
    ra = float(np.float32(p["r_ali"]))
    rsep2, rali2 = np.float32(rs * rs), np.float32(ra * ra)
    w = float(np.float32(weight))
    out = np.zeros((y.shape[0], 3))
    ca = _cells(y, mn, inv, dims)
    for a in range(y.shape[0]):
        acc = np.zeros(3)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    c = ca[a] + np.array([dx, dy, dz])
                    if np.any(c < 0) or np.any(c >= dims):
                        continue
                    key = c[0] + dims[0] * (c[1] + dims[1] * c[2])
                    if cnt[key] == 0:
                        continue
                    centre = mn + (c.astype(np.float32) + np.float32(0.5)) * cell
                    d = centre - y[a]
                    d2 = fp32.dist2(d[0], d[1], d[2])
                    om = 2.0 if d2 < rsep2 else (1.0 if d2 < rali2 else 0.0)
                    acc += om * mean[key]
        out[a] = w * acc
    return out
