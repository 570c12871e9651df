"""Pins of the closure oracle: bfloat16 rounding and GELU against torch's own
routines, gradients against central finite differences, Adam against steps
worked by hand, features against brute-force per-agent binning."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2311_15088_amd import scenes


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0            # tie -> even (down)
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)


def test_gelu_matches_torch_exact_form_and_its_derivative():
    x = np.linspace(-6, 6, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    np.testing.assert_allclose(mlp.gelu(x), ref, rtol=1e-12, atol=1e-15)
    e = 1e-6
    fd = (mlp.gelu(x + e) - mlp.gelu(x - e)) / (2 * e)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def _small_problem(seed=3, B=7):
    rng = np.random.default_rng(seed)
    p = {k: v.astype(np.float64) for k, v in scenes.mlp_init(seed).items()}
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * rng.standard_normal(p[k].shape)
    X = rng.standard_normal((B, 256))
    T = rng.standard_normal((B, 3))
    return p, X, T


def test_forward_matches_torch_float64():
    p, X, _ = _small_problem()
    Y, _ = mlp.forward(p, X, mirror=False)
    t = {k: torch.from_numpy(v) for k, v in p.items()}
    h = torch.nn.functional.gelu(torch.from_numpy(X) @ t["W1"] + t["b1"])
    h = torch.nn.functional.gelu(h @ t["W2"] + t["b2"])
    np.testing.assert_allclose(Y, (h @ t["W3"] + t["b3"]).numpy(), rtol=1e-12, atol=1e-12)


def test_gradients_match_central_differences():
    p, X, T = _small_problem()
    L, g = mlp.loss_and_grads(p, X, T, mirror=False)
    rng = np.random.default_rng(5)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            e = 1e-6 * max(1.0, abs(old))
            flat[idx] = old + e
            lp = mlp.loss_and_grads(p, X, T, mirror=False)[0]
            flat[idx] = old - e
            lm = mlp.loss_and_grads(p, X, T, mirror=False)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * e)
            an = g[k].reshape(-1)[idx]
            # central differences carry ~1e-10 of roundoff in L / e
            assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-9, (k, idx, an, fd)


def test_gradients_match_torch_autograd():
    p, X, T = _small_problem(B=11)
    _, g = mlp.loss_and_grads(p, X, T, mirror=False)
    t = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    h = torch.nn.functional.gelu(torch.from_numpy(X) @ t["W1"] + t["b1"])
    h = torch.nn.functional.gelu(h @ t["W2"] + t["b2"])
    loss = torch.mean((h @ t["W3"] + t["b3"] - torch.from_numpy(T)) ** 2)
    loss.backward()
    for k in p:
        np.testing.assert_allclose(g[k], t[k].grad.numpy(), rtol=1e-10, atol=1e-13)


def test_adam_steps_by_hand():
    # f(w) = w^2 / 2 from w = 1: g = w.  t = 1: m = 0.1, v = 0.001, mh = 1, vh = 1 -> w = 1 - lr
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    lr = 0.1
    mlp.adam_step(p, {"w": p["w"].copy()}, m, v, 1, lr=lr, eps=0.0)
    assert p["w"][0] == pytest.approx(0.9, rel=1e-14)
    # t = 2: g = 0.9; m = 0.09 + 0.09 = 0.18; v = 0.000999 + 0.00081 = 0.001809
    mlp.adam_step(p, {"w": p["w"].copy()}, m, v, 2, lr=lr, eps=0.0)
    mh = 0.18 / (1 - 0.81)
    vh = 0.001809 / (1 - 0.999 ** 2)
    assert p["w"][0] == pytest.approx(0.9 - lr * mh / math.sqrt(vh), rel=1e-12)
    # t = 3 against torch.optim.Adam
    w = torch.tensor([1.0], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    q = {"w": np.array([1.0])}
    mq, vq = {"w": np.zeros(1)}, {"w": np.zeros(1)}
    for t in range(1, 4):
        opt.zero_grad()
        (0.5 * w * w).sum().backward()
        opt.step()
        mlp.adam_step(q, {"w": q["w"].copy()}, mq, vq, t, lr=lr)
    assert q["w"][0] == pytest.approx(w.item(), rel=1e-12)


def test_features_against_brute_force_binning():
    sc = scenes.small_dam(nx=10, ny=8, nz=10, n_agents=9, agents="inside")
    import oracle
    dims, cell, inv, nc = oracle.grid(sc.params)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(sc.x.shape).astype(np.float32)
    f = mlp.features((dims, inv, sc.params["box_min"]), sc.x, v, sc.y, sc.u)
    mn = np.asarray(sc.params["box_min"], np.float32)
    cells = np.clip(np.floor(((sc.x - mn) * np.float32(inv)).astype(np.float32)).astype(int), 0, np.array(dims) - 1)
    for a in range(sc.n_agents):
        c0 = np.rint(((sc.y[a] - mn) * np.float32(inv)).astype(np.float32)).astype(int) - 2
        for q in range(64):
            lx, ly, lz = q % 4, (q // 4) % 4, q // 16
            sel = np.all(cells == c0 + [lx, ly, lz], axis=1)
            n = sel.sum()
            assert f[a, 4 * q] == mlp.bf16_round(n / 8.0)
            if n:
                want = mlp.bf16_round((v[sel].astype(np.float64).mean(0) - sc.u[a]) / 0.5)
                np.testing.assert_array_equal(f[a, 4 * q + 1:4 * q + 4], want)
            else:
                np.testing.assert_array_equal(f[a, 4 * q + 1:4 * q + 4], 0.0)
    assert (f[:, 0::4] > 0).any()


def test_bfloat16_forward_layers_within_their_rounding_error_bounds():
    """Each layer of the bfloat16 forward computes the exact layer of its own
    inputs up to one rounding to bfloat16 (unit roundoff 2^-8, plus 2^-23 for
    the float32 step the rounding goes through) of every input and weight of
    the products, and of every hidden activation after GELU.  The bounds
    are checked element by element; at these sizes they are small next to a
    bias term, so a dropped bias, a missing GELU or a transposed W2 fails."""
    p, X, _ = _small_problem(seed=11, B=64)
    X = 3.0 * X
    for k in ("b1", "b2", "b3"):
        p[k] = 10.0 * p[k]  # biases of order 1
    Y, c = mlp.forward(p, X, mirror=True)
    u = 2.0 ** -8 + 2.0 ** -23
    a = np.abs
    checks = [
        (c["Z1"], X @ p["W1"] + p["b1"], (2 * u + u * u) * (a(X) @ a(p["W1"]))),
        (c["H1"], mlp.gelu(c["Z1"]), u * a(mlp.gelu(c["Z1"]))),
        (c["Z2"], c["H1"] @ p["W2"] + p["b2"], u * (a(c["H1"]) @ a(p["W2"]))),
        (c["H2"], mlp.gelu(c["Z2"]), u * a(mlp.gelu(c["Z2"]))),
        (Y, c["H2"] @ p["W3"] + p["b3"], u * (a(c["H2"]) @ a(p["W3"]))),
    ]
    for k, (got, exact, bound) in enumerate(checks):
        err = a(got - exact)
        assert np.all(err <= bound * (1 + 1e-9) + 1e-12), (k, float((err / (bound + 1e-30)).max()))
    # the roundings act, and the layer bounds are tighter than the terms a slip would drop
    assert a(Y - mlp.forward(p, X, mirror=False)[0]).max() > 0.0
    for k, b in ((2, "b2"), (4, "b3")):
        assert np.median(checks[k][2]) < 0.5 * np.median(a(p[b]))
    assert a(c["H1"] @ p["W2"].T - c["H1"] @ p["W2"]).mean() > 10 * checks[2][2].mean()


def test_bfloat16_gradients_within_their_rounding_error_bounds():
    """The bfloat16 backward rounds the output gradient and each layer's
    pre-activation gradient once to bfloat16 before the products (and uses
    the forward's rounded weights and activations).  Against the exact
    backward of the same forward activations, the gradients of W3 and W2 stay
    within the first-order bound of those roundings, element by element."""
    p, X, T = _small_problem(seed=13, B=64)
    X = 3.0 * X
    B = X.shape[0]
    _, g = mlp.loss_and_grads(p, X, T, mirror=True)
    Y, c = mlp.forward(p, X, mirror=True)
    u = 2.0 ** -8 + 2.0 ** -23
    a = np.abs
    dY = 2.0 * (Y - T) / (3.0 * B)
    # W3: one rounding of dY
    bound3 = u * (a(c["H2"]).T @ a(dY))
    err3 = a(g["W3"] - c["H2"].T @ dY)
    assert np.all(err3 <= bound3 * (1 + 1e-9) + 1e-15)
    # W2: roundings of dY and W3 in the pre-activation gradient, then of that gradient
    gp = mlp.gelu_grad(c["Z2"])
    dZ2 = (dY @ p["W3"].T) * gp
    E = (2 * u + u * u) * (a(dY) @ a(p["W3"]).T) * a(gp)
    bound2 = a(c["H1"]).T @ (E + u * (a(dZ2) + E))
    err2 = a(g["W2"] - c["H1"].T @ dZ2)
    assert np.all(err2 <= bound2 * (1 + 1e-9) + 1e-15)
    assert err2.max() > 0.0 and err3.max() > 0.0
    # tighter than the gradient itself: a wrong operand would not fit
    assert np.median(bound2) < 0.2 * np.median(a(c["H1"].T @ dZ2))
    assert np.median(bound3) < 0.2 * np.median(a(c["H2"].T @ dY))
