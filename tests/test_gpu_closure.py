"""The learned coupling closure on the GPU against the CPU oracle (oracle/mlp.py):
features, the bfloat16 MFMA forward pass, gradients, Adam, training, and the
device-side controller with its fallback to the exact gather."""
import numpy as np
import pytest
import torch

import oracle
import paper_2311_15088_amd as sph
from oracle import mlp
from paper_2311_15088_amd import scenes

from parity import rel_scale_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def bf16_bits(x):
    """float array -> (float64 values rounded to bfloat16, uint16 bit patterns)."""
    r = mlp.bf16_round(x)
    bits = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return r, bits


def to_dev_bits(bits):
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).to(DEV)


def params_np(seed=7):
    rng = np.random.default_rng(seed)
    p = scenes.mlp_init(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = (0.1 * rng.standard_normal(p[k].shape)).astype(np.float32)
    return p


def test_forward_matches_oracle():
    p = params_np()
    rng = np.random.default_rng(1)
    X, bits = bf16_bits(rng.standard_normal((1000, 256)))
    cl = sph.Closure(scenes.mlp_flat(p), force_scale=2.5)
    out = torch.zeros((1000, 3), dtype=torch.float32, device=DEV)
    cl.predict(to_dev_bits(bits), out)
    y, _ = mlp.forward({k: v.astype(np.float64) for k, v in p.items()}, X, mirror=True)
    err = rel_scale_err(out.cpu().numpy(), 2.5 * y)
    print(f"[closure] forward rel err {err:.2e}", flush=True)
    assert err < 2e-3
    cl.close()


def test_gradients_and_loss_match_oracle():
    p = params_np(9)
    rng = np.random.default_rng(2)
    B = 777  # ragged: not a multiple of the 64-row tiles or of 256
    X, bits = bf16_bits(rng.standard_normal((B, 256)))
    F = rng.standard_normal((B, 3)).astype(np.float32)
    scale = 1.7
    cl = sph.Closure(scenes.mlp_flat(p), force_scale=scale)
    g, loss = cl.gradient(to_dev_bits(bits), torch.from_numpy(F).to(DEV))
    L, gref = mlp.loss_and_grads({k: v.astype(np.float64) for k, v in p.items()}, X, F / np.float32(scale))
    assert loss == pytest.approx(L, rel=2e-3)
    gd = scenes.mlp_unflat(g)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        err = rel_scale_err(gd[k].reshape(len(gd[k]), -1), gref[k].reshape(len(gref[k]), -1))
        print(f"[closure] grad {k} rel err {err:.2e}", flush=True)
        assert err < 2e-3, k
    cl.close()


def test_adam_step_matches_oracle():
    p = params_np(11)
    rng = np.random.default_rng(3)
    cl = sph.Closure(scenes.mlp_flat(p))
    ref = {k: v.astype(np.float64) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in ref.items()}
    v = {k: np.zeros_like(v) for k, v in ref.items()}
    for t in range(1, 4):
        g = (1e-2 * rng.standard_normal(sph.CLOSURE_PARAMS)).astype(np.float32)
        cl.adam_step(g, t, lr=1e-3)
        mlp.adam_step(ref, {k: val.astype(np.float64) for k, val in scenes.mlp_unflat(g).items()}, m, v, t, lr=1e-3)
    w, _ = cl.weights()
    np.testing.assert_allclose(w, scenes.mlp_flat({k: val.astype(np.float32) for k, val in ref.items()}),
                               rtol=1e-5, atol=1e-8)
    cl.close()


def test_features_match_oracle():
    sc = scenes.small_dam(nx=14, ny=10, nz=14, n_agents=40, agents="inside")
    rng = np.random.default_rng(4)
    v = (0.3 * rng.standard_normal(sc.x.shape)).astype(np.float32)
    sim = sph.Simulation(sc.params, sc.x, v, sc.y, sc.u, flags=sph.FLAG_FEATURES)
    sim.step(1)
    f = sim.read(sph.AGENT_FEATURES)  # features of the state the step started from
    dims, cell, inv, nc = oracle.grid(sc.params)
    ref = mlp.features((dims, inv, sc.params["box_min"]), sc.x, v, sc.y, sc.u)
    got = (f.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    # float32 vs float64 means may round to neighbouring bfloat16 values
    ulp = np.maximum(np.abs(ref), 1e-30) * 2.0 ** -7
    assert np.all(np.abs(got - ref) <= ulp + 1e-12)
    assert np.mean(got == ref) > 0.99
    sim.close()


def _collect(sc, steps):
    sim = sph.Simulation(sc.params, sc.x, sc.v, sc.y, sc.u, flags=sph.FLAG_FEATURES | sph.FLAG_DIAGNOSTICS)
    feats, forces = [], []
    for _ in range(steps):
        sim.step(1)
        feats.append(sim.read(sph.AGENT_FEATURES))
        forces.append(sim.read(sph.AGENT_FORCE))
    sim.close()
    return np.concatenate(feats), np.concatenate(forces)


def test_training_lowers_error_and_controller_switches():
    sc = scenes.dam_break("agents", 24, 12, 24, 0.05, (0, 0, 0), (1.2, 0.6, 1.2), 4000, 5e-4, 10,
                          scenes.SEED0 + 0x901, agents="inside")
    feats, forces = _collect(sc, 6)
    print(f"[closure] {len(feats)} training pairs", flush=True)
    cl = sph.Closure(scenes.mlp_flat(scenes.mlp_init()))
    F = torch.from_numpy(forces.astype(np.float32)).to(DEV)
    X = to_dev_bits(feats)
    rep0 = cl.train(X, F, epochs=0, batch=1024, val_fraction=0.2, seed=1)
    rep = cl.train(X, F, epochs=30, batch=1024, val_fraction=0.2, seed=1)
    print(f"[closure] untrained val rel rms {rep0['val_rel_rms']:.3f}, trained {rep['val_rel_rms']:.3f}", flush=True)
    assert rep["val_rel_rms"] < 0.8 * rep0["val_rel_rms"]
    # controller: a bound of 0 always falls back -> identical to the exact run
    a = sph.create(sc)
    a.attach_closure(cl, check_every=3, max_rel_rms=0.0)
    a.step(7)
    st = a.closure_stats()
    assert st["checks"] == 3 and st["fallbacks"] == 3 and st["surrogate_steps"] == 0 and st["exact_steps"] == 7
    b = sph.create(sc)
    b.step(7)
    for f in (sph.POS, sph.VEL, sph.AGENT_POS, sph.AGENT_VEL):
        np.testing.assert_array_equal(a.read(f), b.read(f))
    # an unbounded threshold switches to the surrogate after the first check
    c = sph.create(sc)
    c.attach_closure(cl, check_every=3, max_rel_rms=1e30)
    c.step(7)
    st = c.closure_stats()
    assert st["mode"] == 1 and st["checks"] == 3 and st["surrogate_steps"] == 4 and st["exact_steps"] == 3
    c.attach_closure(None)
    for s in (a, b, c):
        s.close()
    cl.close()


def _step_matches_predict(sim, cl):
    """fhat of the last step (fused in-step inference) against Closure.predict on
    the same features: bit-identical where the agent's block holds fluid, 0 elsewhere."""
    feats = sim.read(sph.AGENT_FEATURES)
    fhat = sim.read(sph.AGENT_FORCE_MODEL)
    pred = torch.zeros((feats.shape[0], 3), dtype=torch.float32, device=DEV)
    cl.predict(to_dev_bits(feats), pred)
    pred = pred.cpu().numpy()
    occ = (feats[:, 0::4] != 0).any(axis=1)
    assert occ.any() and not occ.all()
    want = np.where(occ[:, None], pred, np.float32(0.0))
    np.testing.assert_array_equal(fhat.view(np.uint32), want.view(np.uint32))


def test_in_step_inference_equals_predict():
    # agents in the upper half of the box: some blocks hold fluid, some do not;
    # a ragged count (not a multiple of 16 or 64)
    sc = scenes.dam_break("agents", 24, 12, 24, 0.05, (0, 0, 0), (1.2, 0.6, 1.2), 1001, 5e-4, 10,
                          scenes.SEED0 + 0x907, agents="upper")
    cl = sph.Closure(scenes.mlp_flat(params_np(11)), force_scale=2.5)
    sim = sph.create(sc)
    sim.attach_closure(cl, check_every=2, max_rel_rms=1e30)
    sim.step(3)
    assert sim.closure_stats()["surrogate_steps"] >= 1
    _step_matches_predict(sim, cl)
    # changed weights (an Adam step, then a direct write) reach the in-step copy
    feats = sim.read(sph.AGENT_FEATURES)
    target = np.random.default_rng(5).standard_normal((feats.shape[0], 3)).astype(np.float32)
    g, _ = cl.gradient(to_dev_bits(feats), torch.from_numpy(target).to(DEV))
    cl.adam_step(g, 1, lr=1e-2)
    sim.step(1)
    _step_matches_predict(sim, cl)
    w, _ = cl.weights()
    cl.set_weights(0.5 * w, force_scale=0.75)
    sim.step(1)
    _step_matches_predict(sim, cl)
    sim.attach_closure(None)
    sim.close()
    cl.close()


def test_gain_of_the_trained_network_on_config4():
    """What the trained network gains over the method without it, on the
    4,194,304-particle / 65,536-agent workload: trained on this project's GPU
    kernels with pairs from config-4-style runs of another seed, then measured
    against the exact per-agent gather on the workload itself.

    Measured (and asserted): the trained network's relative RMS force error
    is well below that of predicting nothing (1.0) and of the untrained
    network, but far above the 2 % bound, so the controller keeps the exact
    gather at every check and the step is bit-identical to the exact one; the
    surrogate path's time is measured beside the exact gather's."""
    dev = torch.device(DEV)
    train_sc = scenes.dam_break("c4", 256, 64, 256, 0.02, (0, 0, 0), (3, 1, 3), 65536, 2e-4, 100,
                                scenes.SEED0 + 0x410, agents="inside")
    sim = sph.create(train_sc, flags=sph.FLAG_FEATURES | sph.FLAG_DIAGNOSTICS)
    X = torch.empty((6 * 65536, 256), dtype=torch.int16, device=dev)
    F = torch.empty((6 * 65536, 3), dtype=torch.float32, device=dev)
    for k in range(6):
        sim.step(4)
        sim.read_into(sph.AGENT_FEATURES, X[k * 65536:(k + 1) * 65536])
        sim.read_into(sph.AGENT_FORCE, F[k * 65536:(k + 1) * 65536])
    sim.close()
    del train_sc
    cl = sph.Closure(scenes.mlp_flat(scenes.mlp_init()))
    untrained = sph.Closure(scenes.mlp_flat(scenes.mlp_init()))
    rep = cl.train(X, F, epochs=8, batch=4096, lr=1e-3, val_fraction=0.1, seed=3)
    untrained_rep = untrained.train(X, F, epochs=0, batch=4096, val_fraction=0.1, seed=3)  # sets the force scale only
    del X, F
    print(f"[closure] trained on {6 * 65536} pairs: {rep}", flush=True)
    # the workload itself: exact force and features of a few steps
    sc = scenes.config4()
    sim = sph.create(sc, flags=sph.FLAG_FEATURES | sph.FLAG_DIAGNOSTICS)
    num = {"trained": 0.0, "untrained": 0.0}
    den = 0.0
    for _ in range(3):
        sim.step(5)
        feats = torch.empty((sc.n_agents, 256), dtype=torch.int16, device=dev)
        exact = torch.empty((sc.n_agents, 3), dtype=torch.float32, device=dev)
        sim.read_into(sph.AGENT_FEATURES, feats)
        sim.read_into(sph.AGENT_FORCE, exact)
        for name, net in (("trained", cl), ("untrained", untrained)):
            pred = torch.empty_like(exact)
            net.predict(feats, pred)
            num[name] += float(((pred.double() - exact.double()) ** 2).sum())
        den += float((exact.double() ** 2).sum())
    sim.close()
    err = {k: (v / den) ** 0.5 for k, v in num.items()}
    print(f"[closure] config 4 rel RMS: trained {err['trained']:.3f}, untrained {err['untrained']:.3f}, "
          f"predicting nothing 1.000", flush=True)
    assert err["trained"] < 0.9 and err["trained"] < 0.9 * err["untrained"]
    # time: the agent phase with the exact gather, and with the surrogate path forced
    times = {}
    for name, bound in (("exact", None), ("surrogate", 1e30), ("controller", 0.02)):
        s = sph.create(sc)
        if bound is not None:
            s.attach_closure(cl, check_every=50, max_rel_rms=bound)
        s.step(2)
        ph = s.step_profiled(20)
        times[name] = 1e3 * ph["agents"] / 20
        if name == "controller":
            st = s.closure_stats()
            print(f"[closure] controller at 2 %: {st}", flush=True)
            assert st["checks"] >= 1 and st["fallbacks"] == st["checks"] and st["surrogate_steps"] == 0
            ref = sph.create(sc)
            ref.step(22)
            for f in (sph.POS, sph.VEL, sph.AGENT_POS, sph.AGENT_VEL):
                np.testing.assert_array_equal(s.read(f), ref.read(f))
            ref.close()
        if bound is not None:
            s.attach_closure(None)
        s.close()
    print(f"[closure] agents phase us/step: exact {times['exact']:.1f}, surrogate path {times['surrogate']:.1f}, "
          f"under the 2 % controller {times['controller']:.1f}", flush=True)
    assert all(t > 0 for t in times.values())
    cl.close()
    untrained.close()


def test_checkpoint_of_weights_and_adam_moments_resumes_bit_identically():
    """sph_closure_io saves weights, both Adam moments, the force scale and the
    step count; a closure loaded from it continues the optimiser exactly as
    the original does."""
    rng = np.random.default_rng(8)
    _, bits = bf16_bits(rng.standard_normal((500, 256)))
    X = to_dev_bits(bits)
    T = torch.from_numpy(rng.standard_normal((500, 3)).astype(np.float32)).to(DEV)
    a = sph.Closure(scenes.mlp_flat(params_np(13)), force_scale=1.3)
    for t in (1, 2, 3):
        g, _ = a.gradient(X, T)
        a.adam_step(g, t, lr=1e-2)
    state = a.save_state()
    assert state.size == sph.CLOSURE_STATE_FLOATS and state[-1] == 3.0 and state[-2] == np.float32(1.3)
    assert np.abs(state[sph.CLOSURE_PARAMS:2 * sph.CLOSURE_PARAMS]).max() > 0  # first moments are there
    b = sph.Closure(None)
    b.load_state(state)
    np.testing.assert_array_equal(b.save_state(), state)
    for cl in (a, b):
        for t in (4, 5):
            g, _ = cl.gradient(X, T)
            cl.adam_step(g, t, lr=1e-2)
    wa, sa = a.weights()
    wb, sb = b.weights()
    np.testing.assert_array_equal(wa, wb)
    np.testing.assert_array_equal(a.save_state(), b.save_state())
    bad = state.copy()
    bad[-2] = 0.0  # force scale must be positive
    with pytest.raises(sph.SphError) as ei:
        b.load_state(bad)
    assert ei.value.status == sph.EINVAL
    a.close()
    b.close()
