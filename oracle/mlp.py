"""CPU reference for the learned coupling closure (test infrastructure only).

The closure maps each agent's neighbourhood histogram to its fluid coupling
force.  Features: the 4 x 4 x 4 block of fluid-grid cells starting at
c0 = round(fl32(fl32(y - min) * inv_d)) - 2 on every axis; per cell (x
fastest, then y, then z) the count / 8 and the mean fluid velocity minus the
agent's velocity, divided by 0.5 (zero for an empty or out-of-grid cell):
64 cells x 4 values = 256 features, rounded to bfloat16.

Network: 256 -> 128 -> 128 -> 3 with GELU (x Phi(x), the erf form) after the
two hidden layers.  Matrix products take bfloat16 operands (weights, inputs,
activations; round-to-nearest-even) and accumulate exactly (float64 here,
float32 on the GPU).  The backward pass rounds the upstream gradient of each
layer to bfloat16 before its products, like the GPU kernels.  Loss: mean
squared error over the three output components of a batch, on forces divided
by a fixed scale.  Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on
float64 master weights here (float32 on the GPU).

Only tests/, the smoke check and the bench's CPU baseline may use this module.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

try:
    from scipy.special import erf as _erf
except Exception:  # pragma: no cover
    _erf = np.vectorize(math.erf)

SIZES = (256, 128, 128, 3)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out = np.where(nan, np.nan, out)
    return out


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(p: Dict[str, np.ndarray], X, mirror: bool = True) -> Tuple[np.ndarray, Dict]:
    """Outputs [B, 3] and the activations the backward pass needs."""
    r = bf16_round if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    X0 = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    Z1 = X0 @ W1 + p["b1"]
    H1 = r(gelu(Z1))
    Z2 = H1 @ W2 + p["b2"]
    H2 = r(gelu(Z2))
    Y = H2 @ W3 + p["b3"]
    return Y, dict(X0=X0, Z1=Z1, H1=H1, Z2=Z2, H2=H2, W1=W1, W2=W2, W3=W3)


def loss_and_grads(p: Dict[str, np.ndarray], X, T, mirror: bool = True):
    """MSE over all output components and its gradient with respect to p."""
    r = bf16_round if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    Y, c = forward(p, X, mirror)
    T = np.asarray(T, dtype=np.float64)
    B = Y.shape[0]
    L = float(np.mean((Y - T) ** 2))
    dY = 2.0 * (Y - T) / (3.0 * B)
    g = {}
    dYb = r(dY)
    g["W3"] = c["H2"].T @ dYb
    g["b3"] = dY.sum(0)
    dZ2 = (dYb @ c["W3"].T) * gelu_grad(c["Z2"])
    dZ2b = r(dZ2)
    g["W2"] = c["H1"].T @ dZ2b
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2b @ c["W2"].T) * gelu_grad(c["Z1"])
    dZ1b = r(dZ1)
    g["W1"] = c["X0"].T @ dZ1b
    g["b1"] = dZ1.sum(0)
    return L, g


def adam_step(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); updates p, m, v in place."""
    for k in p:
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def features(grid, x, v, y, u) -> np.ndarray:
    """Per-agent features [A, 256] (float64, already rounded to bfloat16).

    grid: (dims, inv_d, box_min) of the fluid grid, as the oracle's grid().
    """
    dims, inv, bmin = grid
    x = np.asarray(x, np.float32)
    v = np.asarray(v, np.float64)
    y = np.asarray(y, np.float32)
    u = np.asarray(u, np.float64)
    mn = np.asarray(bmin, np.float32)
    inv32 = np.float32(inv)
    dims = np.asarray(dims, np.int64)
    # fluid cells (floor, clamped) and per-cell count / velocity sums
    t = ((x - mn).astype(np.float32) * inv32).astype(np.float32)
    c = np.clip(np.floor(t).astype(np.int64), 0, dims - 1)
    key = c[:, 0] + dims[0] * (c[:, 1] + dims[1] * c[:, 2])
    ncell = int(np.prod(dims))
    cnt = np.bincount(key, minlength=ncell).astype(np.float64)
    vs = np.stack([np.bincount(key, weights=v[:, k], minlength=ncell) for k in range(3)], axis=1)
    # agent blocks
    ta = ((y - mn).astype(np.float32) * inv32).astype(np.float32)
    c0 = np.rint(ta).astype(np.int64) - 2
    A = y.shape[0]
    out = np.zeros((A, 64, 4))
    for lz in range(4):
        for ly in range(4):
            for lx in range(4):
                q = lx + 4 * (ly + 4 * lz)
                cc = c0 + np.array([lx, ly, lz])
                inside = np.all((cc >= 0) & (cc < dims), axis=1)
                k = cc[:, 0] + dims[0] * (cc[:, 1] + dims[1] * cc[:, 2])
                k = np.where(inside, k, 0)
                n = np.where(inside, cnt[k], 0.0)
                out[:, q, 0] = n / 8.0
                has = n > 0
                mean = np.where(has[:, None], vs[k] / np.maximum(n, 1.0)[:, None], 0.0)
                out[:, q, 1:] = np.where(has[:, None], (mean - u) / 0.5, 0.0)
    return bf16_round(out.reshape(A, 256))


def rel_rms(pred, exact) -> float:
    """sqrt(sum |pred - exact|^2 / sum |exact|^2) over all agents."""
    pred = np.asarray(pred, np.float64)
    exact = np.asarray(exact, np.float64)
    den = np.sum(exact * exact)
    return float(np.sqrt(np.sum((pred - exact) ** 2) / den)) if den > 0 else 0.0
