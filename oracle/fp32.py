"""Single-precision arithmetic the oracle's numpy modules need exactly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The squared-distance predicate of every neighbourhood decision is evaluated
in float32 as fl(dz * dz + fl(dy * dy + fl(dx * dx))), each of the two outer
steps a fused multiply-add (one rounding of the exact product-plus-sum), with
dx = fl(x_j - x_i) per axis.  numpy has no fused multiply-add, so
``fmaf32`` forms it exactly: the float32 operands' product is exact in
float64 (24 + 24 bits), the float64 sum is made exact by Knuth's TwoSum, and
the exact result is rounded to float32 through round-to-odd at double
precision (Boldo and Melquiond, "Emulation of FMA and correctly rounded sums:
proved algorithms using rounding to odd", IEEE Trans. Computers 2008): the
truncated double with its last bit set when inexact rounds to the same
float32 as the exact value, because double keeps more than 24 + 1 bits.
"""
from __future__ import annotations

import numpy as np


def fmaf32(a, b, c) -> np.ndarray:
    """float32 round-to-nearest-even of a * b + c, computed exactly."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b                       # exact
    s = np.asarray(p + c, np.float64)
    bb = s - p
    err = np.asarray((p - (s - bb)) + (c - bb), np.float64)  # p + c = s + err exactly
    # truncate p + c toward zero at double precision ...
    grows = np.sign(err) == np.sign(s)  # |p + c| > |s|: s is already the truncation
    t = np.where(err == 0.0, s, np.where(grows, s, np.nextafter(s, 0.0)))
    # ... and mark it inexact in its last bit (round to odd)
    odd = t.view(np.uint64) | np.where(err != 0.0, np.uint64(1), np.uint64(0))
    return odd.view(np.float64).astype(np.float32)


def dist2(dx, dy, dz) -> np.ndarray:
    """fl(dz^2 + fl(dy^2 + fl(dx^2))) with the two outer steps fused."""
    dx = np.asarray(dx, np.float32)
    dy = np.asarray(dy, np.float32)
    dz = np.asarray(dz, np.float32)
    return fmaf32(dz, dz, fmaf32(dy, dy, (dx * dx).astype(np.float32)))
