"""Materialised neighbour lists, as the paper's list-based neighbour search
defines them -- the reference for the library's list forms.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy; the cell
keys and the (key, id) order come from the C oracle's step.

"Neighbor Search with Sorting" section: after the counting sort, every
particle's list holds the particles of the 27 cells around its own cell
whose squared distance to it is below h^2, found by walking those cells in
the sorted array.  The predicate is the single-precision one of the oracle:
dx = fl(x_j - x_i) per axis, then fl(dz^2 + fl(dy^2 + fl(dx^2))) with the two
outer steps fused multiply-adds (``oracle/fp32.py``), against h^2 = fl32(h * h)
with h the float32 parameter in double.

Reading of this project (the paper lists neighbours but does not fix their
order or whether i itself is kept): each list includes the particle itself
(r^2 = 0 < h^2, the self term of the density) and is ordered by halo row
(dz, then dy, each in -1, 0, 1) and, within a row, by sorted index -- the
three cells of a row are consecutive in the sorted array.  Entries are sorted
indices.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np

from . import fp32, grid, step


def sorted_state(p: Dict, x) -> Dict[str, np.ndarray]:
    """The (key, id) order of one step from the float32 positions: sorted ids,
    the cell key and the integer cell coordinates of each sorted particle."""
    x = np.ascontiguousarray(np.asarray(x, np.float32)).reshape(-1, 3)
    none = np.zeros((0, 3), np.float32)
    r = step(p, x, np.zeros_like(x), none, none, fsample=np.zeros(0, np.int64), asample=np.zeros(0, np.int64))
    dims = grid(p, False)[0]
    order = r["sorted"].astype(np.int64)
    key = r["key"][order].astype(np.int64)
    c = np.stack([key % dims[0], (key // dims[0]) % dims[1], key // (dims[0] * dims[1])], axis=1)
    return dict(order=order, key=key, cell=c, xs=x[order], dims=np.asarray(dims))


def neighbour_lists(p: Dict, x) -> List[np.ndarray]:
    """lists[i]: the sorted indices j in the list of sorted particle i."""
    st = sorted_state(p, x)
    xs, c = st["xs"], st["cell"]
    h = float(np.float32(p["h"]))
    h2 = np.float32(h * h)
    out = []
    for i in range(xs.shape[0]):
        d = c - c[i]
        # the 27 cells around i's cell: every axis within one cell
        cand = np.nonzero(np.all(np.abs(d) <= 1, axis=1))[0]
        dx = xs[cand, 0] - xs[i, 0]
        dy = xs[cand, 1] - xs[i, 1]
        dz = xs[cand, 2] - xs[i, 2]
        r2 = fp32.dist2(dx, dy, dz)  # float32, the outer two steps fused
        keep = cand[r2 < h2]
        # halo row (dz, dy), then sorted index
        row = (d[keep, 2] + 1) * 3 + (d[keep, 1] + 1)
        out.append(keep[np.lexsort((keep, row))].astype(np.uint32))
    return out
