#!/usr/bin/env python3
"""Benchmark: SPH + boid time steps on one MI355X.

Workload: the 1,048,576-particle dam break (128 x 64 x 128 lattice, s = 0.01,
h = 0.02, box [0,3] x [0,1] x [0,3]) with 1,024 boid agents above the fluid,
dt = 2e-4 -- seeded synthetic inputs, already resident in HBM when timing
starts.  A step is one pass of the whole path: cell keys + counting sort,
density, boid steering + coupling, forces + integration.

Three regions run the same K steps from the same initial state:
  * timed region: K steps launched directly on the library's stream, with
    HIP events only at the density and force kernels' own start and end (the
    whole-step time, `value`, and the dominant kernel's duration for the
    roofline come from this region);
  * phase region: the same K steps with an event between every two phases
    as well (the per-phase breakdown; the extra events cost some time
    between launches, so its step time is reported but not used);
  * graph region: K steps replayed from captured HIP graphs, without events
    (reported beside).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed
# dual issue) x 2.4 GHz.  This code is built without packed FP32, so half of
# it (78.6 TFLOP/s) is the attainable ceiling; the published figure is the peak.
PEAK_FP32_TFLOPS = 157.3

# Algorithmic FP32 operations of the force + integration pass: per neighbour
# pair (i, j in N_i) the pair term of the pressure and viscosity forces
# (displacement 3, r^2 5, cut-off test 1, r, q, w 3, pressure coefficient 5,
# velocity difference and viscosity coefficient 4, pair vector 13, sum 3), and
# per particle the division by rho, coupling scale, gravity, Euler-Cromer
# update and walls.
FLOP_FORCE_PER_PAIR = 37
FLOP_FORCE_PER_PARTICLE = 30

# HBM traffic of one force + integration launch from two rocprofv3 counter
# runs (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the scale factors a plain
# 1 GiB device copy reads on the same counters), averaged over the 1,000 steps
# this script times; valid only for the kernel sources it was measured on.
TRAFFIC_FORCE = {"sources_sha256_16": "202bf95d776f86b3", "bytes_per_launch": 315.4e6,
                 "measured_on": "the 1,000 timed steps"}
FORCE_SOURCES = ("paper_2311_15088_amd/csrc/sph_fluid_impl.hpp", "paper_2311_15088_amd/csrc/sph_physics.hip")


def force_traffic():
    import hashlib

    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_FORCE["bytes_per_launch"] if h.hexdigest()[:16] == TRAFFIC_FORCE["sources_sha256_16"] else None

# Algorithmic bytes per element and launch for each kernel of a step (the
# arrays each kernel must read and write once, in the layout it uses).
#   key_count      reads x,y,z (12), writes key, rank (8)             per particle
#   scan_reduce    reads cnt (4)                                       per cell
#   scan_apply     reads cnt (4), writes off (4), clears cnt (4)       per cell
#   scatter        reads key, rank, id (12), writes src, id (8)        per particle
#   fixup_tile_list reads src, id, key (12), x, v (24), writes x, v, id (28) per particle
#                  (the work-item list in the same launch: 8 per tile)
#   density        reads x (12), writes rho, n (8)                     per particle
#   force_integrate reads x, v, rho (28), writes x', v' (24)           per particle
#   agents         reads y, u (24), writes y', u' (24)                 per agent
B_PER_PARTICLE = {"key_count": 20, "scatter": 20, "fixup_tile_list": 64, "density": 20, "force_integrate": 52}
B_PER_CELL = {"scan_reduce": 4, "scan_apply": 12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name, n, cells, agents):
    if name in B_PER_PARTICLE:
        return B_PER_PARTICLE[name] * n
    if name in B_PER_CELL:
        return B_PER_CELL[name] * cells
    if name == "agents":
        return 48 * agents
    return 0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(sc, budget_s: float):
    """The CPU oracle timed on the host cores on whole steps of the same workload."""
    import oracle  # test infrastructure: only this leg of the bench uses it

    x, v, y, u = sc.x, sc.v, sc.y, sc.u
    steps = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.step(sc.params, x, v, y, u, nbr_mode=1)
        x, v = r["x1"].astype(np.float32), r["v1"].astype(np.float32)
        y, u = r["y1"].astype(np.float32), r["u1"].astype(np.float32)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    return {
        "value": steps * sc.n / el, "unit": "particle-steps/s", "cores": oracle.threads(), "kind": "oracle",
        "sample": f"{steps} whole step(s) of the same {sc.n}-particle workload from its initial state, FP64 "
                  f"oracle with its cell-list neighbour finder (sets identical to brute force), "
                  f"{oracle.threads()} OpenMP threads on '{cpu_model()}', {el:.1f} s",
    }


def scale_leg(sph, scenes, torch, args):
    """16,777,216 particles in two unequal blocks, 2^24 cells, 65,536 agents in flocks."""
    sc = scenes.config2()
    log(f"[bench] scale: n={sc.n} agents={sc.n_agents}")
    stream = torch.cuda.current_stream().cuda_stream
    sim = sph.create(sc, stream=stream)
    K = args.scale_steps
    sim.step_timed(25)
    torch.cuda.synchronize()
    pairs0 = int(sim.read(sph.PAIR_COUNT)[0])
    t0 = time.perf_counter()
    ph = sim.step_timed(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = int(sim.read(sph.PAIR_COUNT)[0]) - pairs0
    info = sim.info()
    sim.close()
    b_alg = 154.0 + 24.0 * info["cells"] / sc.n
    ms = 1e3 * wall / K
    return {"workload": "two blocks 128x256x384 + 128x256x128 = 16,777,216 particles + 65,536 boids, h=0.01, "
                        "dt=1e-4, 2^24 cells", "steps": K, "ms_per_step": ms,
            "particle_steps_per_s": sc.n * K / wall, "pair_interactions_per_s": pairs / wall,
            "mean_neighbours": pairs / (K * sc.n), "step_hbm_frac": b_alg * sc.n / (ms * 1e-3) / (PEAK_HBM_GBS * 1e9),
            "kernel_us_per_step": {k: 1e3 * v / K for k, v in ph.items()}}


def search_leg(sph, scenes, torch, args):
    """The paper's list-based neighbour searches against the tiled gather on the
    same workload: per-phase times, with the sort plus the list build taken as
    the neighbour search."""
    sc = scenes.config1()
    stream = torch.cuda.current_stream().cuda_stream
    K = args.search_steps
    out = {"workload": "dam break 128x64x128 = 1,048,576 particles + 1,024 boids, h=0.02, dt=2e-4", "steps": K}
    names = {sph.SEARCH_TILES: "tiled_gather", sph.SEARCH_SORTED_LIST: "sorted_list",
             sph.SEARCH_BUCKET_LIST: "bucket_list"}
    search_phases = ("key_count", "scan_reduce", "scan_apply", "scatter", "fixup_tile_list")
    for mode, name in names.items():
        sim = sph.create(sc, stream=stream)
        if mode != sph.SEARCH_TILES:
            sim.set_search(mode)
        sim.step_profiled(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = sim.step_profiled(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        us = {k: 1e3 * v / K for k, v in ph.items()}
        out[name] = {"ms_per_step": 1e3 * wall / K, "us_per_step": us,
                     "neighbour_search_us": sum(us[k] for k in search_phases),
                     "fluid_passes_us": us["density"] + us["force_integrate"]}
        log(f"[bench] search {name}: {1e3 * wall / K:.4f} ms/step, neighbour search "
            f"{out[name]['neighbour_search_us']:.1f} us, density + force {out[name]['fluid_passes_us']:.1f} us")
    return out


def voxel_leg(sph, scenes, torch, args):
    """Voxel density at cube corners on the 1M-particle workload (corner spacing
    h/2, neighbourhood radius h, particle radius h/4): the step with and without
    the voxel kernel (the phase events time the density kernel itself, so the
    voxel kernel shows in the step time)."""
    sc = scenes.config1()
    h = sc.params["h"]
    stream = torch.cuda.current_stream().cuda_stream
    K = args.search_steps
    out = {"workload": "dam break 128x64x128 = 1,048,576 particles, box 3x1x3, corners every h/2, R = h, r = h/4",
           "steps": K}
    for on in (False, True):
        sim = sph.create(sc, stream=stream)
        if on:
            out["corners"] = int(np.prod(sim.enable_voxels(0.5 * h, h, 0.25 * h)))
        sim.step_profiled(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = sim.step_profiled(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        out["with_voxels" if on else "without"] = {"ms_per_step": 1e3 * wall / K,
                                                    "density_phase_us": 1e3 * ph["density"] / K}
    us = 1e3 * (out["with_voxels"]["ms_per_step"] - out["without"]["ms_per_step"])
    out["voxel_us_per_step"] = us
    out["corners_per_s"] = out["corners"] / (us * 1e-6) if us > 0 else None
    log(f"[bench] voxel: {out['corners']} corners, {us:.1f} us per field")
    return out


def obstacle_leg(sph, scenes, torch, args):
    """Obstacle avoidance on the 1M-particle workload: two boxes in the boids'
    region (the agent phase with and without the obstacle term)."""
    sc = scenes.config1()
    lo, hi = sc.y.min(0), sc.y.max(0)
    ext = hi - lo
    boxes = np.array([np.concatenate([lo + 0.2 * ext, lo + 0.4 * ext]),
                      np.concatenate([lo + 0.6 * ext, lo + 0.8 * ext])], np.float32)
    stream = torch.cuda.current_stream().cuda_stream
    K = args.search_steps
    out = {"workload": "dam break 1,048,576 particles + 1,024 boids, two boxes among the boids, vertices every h",
           "steps": K}
    for on in (False, True):
        sim = sph.create(sc, stream=stream)
        if on:
            sim.set_obstacles(boxes, sc.params["h"], 1.0)
        sim.step_profiled(10)
        torch.cuda.synchronize()
        ph = sim.step_profiled(K)
        torch.cuda.synchronize()
        sim.close()
        out["with_obstacles_agents_us" if on else "without_agents_us"] = 1e3 * ph["agents"] / K
    log(f"[bench] obstacles: agents phase {out['without_agents_us']:.2f} -> {out['with_obstacles_agents_us']:.2f} us")
    return out


def batched_leg(sph, scenes, torch, args):
    """512 independent dam breaks of uneven size: one batched context vs a loop of plain steps."""
    scs = scenes.batched(args.scenes)
    n_tot = sum(s.n for s in scs)
    log(f"[bench] batched: {len(scs)} scenes, {n_tot} particles, {sum(s.n_agents for s in scs)} agents")
    stream = torch.cuda.current_stream().cuda_stream
    bat = sph.create_batch(scs, stream=stream)
    tuned = bat.autotune(2)
    log(f"[bench] batched autotune: {tuned}")
    K = args.batched_steps
    bat.step(2)
    bat.capture(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bat.step(K)  # one graph of K steps
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    bat.close()
    # a loop of plain steps, one scene after another (K_plain steps each)
    Kp = max(1, K // 10)
    tp = 0.0
    for sc in scs:
        sim = sph.create(sc, stream=stream)
        sim.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(Kp)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        sim.close()
    return {
        "scenes": len(scs), "particles": n_tot, "steps": K,
        "scene_steps_per_s": len(scs) * K / tb, "particle_steps_per_s": n_tot * K / tb,
        "plain_loop_scene_steps_per_s": len(scs) * Kp / tp, "plain_loop_steps_per_scene": Kp,
        "speedup_vs_plain_loop": (len(scs) * K / tb) / (len(scs) * Kp / tp),
        "autotuned": tuned,
    }


def closure_leg(sph, scenes, torch, args):
    """Learned coupling closure on the 4,194,304-particle / 65,536-agent workload."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    # training pairs from config-4-style runs with other seeds
    want = args.pairs
    X = torch.empty((want, 256), dtype=torch.int16, device=dev)
    F = torch.empty((want, 3), dtype=torch.float32, device=dev)
    got, seed = 0, 1
    t0 = time.perf_counter()
    while got < want:
        sc = scenes.dam_break("c4", 256, 64, 256, 0.02, (0, 0, 0), (3, 1, 3), 65536, 2e-4, 100,
                              scenes.SEED0 + 0x400 + 0x10 * seed, agents="inside")
        sim = sph.create(sc, stream=stream, flags=sph.FLAG_FEATURES | sph.FLAG_DIAGNOSTICS)
        for _ in range(16):
            if got >= want:
                break
            sim.step(5)
            take = min(sc.n_agents, want - got)
            xs = torch.empty((sc.n_agents, 256), dtype=torch.int16, device=dev)
            fs = torch.empty((sc.n_agents, 3), dtype=torch.float32, device=dev)
            sim.read_into(sph.AGENT_FEATURES, xs)
            sim.read_into(sph.AGENT_FORCE, fs)
            X[got:got + take] = xs[:take]
            F[got:got + take] = fs[:take]
            got += take
        sim.close()
        seed += 1
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    log(f"[bench] closure: collected {got} pairs in {t_collect:.1f} s")
    cl = sph.Closure(scenes.mlp_flat(scenes.mlp_init()), stream=stream)
    rep = cl.train(X, F, epochs=args.epochs, batch=4096, lr=1e-3, val_fraction=0.1, seed=7)
    log(f"[bench] closure: trained {rep}")
    del X, F
    # evaluation run: the workload itself, exact gather vs closure
    sc = scenes.config4()
    K = args.closure_steps
    res = {"pairs": got, "collect_s": t_collect, "train": rep, "steps": K}
    # exact gather; the closure under its controller (2 % bound, check every
    # 50 steps); the closure with an unbounded threshold, which times the
    # surrogate path whatever its error
    for name, attach, bound in (("exact", False, 0.0), ("closure", True, 0.02), ("surrogate_forced", True, 1e30)):
        sim = sph.create(sc, stream=stream)
        if attach:
            sim.attach_closure(cl, check_every=50, max_rel_rms=bound)
        ph = sim.step_profiled(K)
        res[name] = {"agents_us_per_step": 1e3 * ph["agents"] / K, "ms_per_step": sum(ph.values()) / K}
        if attach:
            res[name]["stats"] = sim.closure_stats()
            sim.attach_closure(None)
        sim.close()
    res["coupling_speedup"] = res["exact"]["agents_us_per_step"] / res["closure"]["agents_us_per_step"]
    res["coupling_speedup_surrogate_path"] = (res["exact"]["agents_us_per_step"] /
                                              res["surrogate_forced"]["agents_us_per_step"])
    cl.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--chunk", type=int, default=50, help="steps per captured graph in the graph region")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--scale", action="store_true", help="add the 16.7M-particle scale workload")
    ap.add_argument("--scale-steps", type=int, default=200)
    ap.add_argument("--batched", action="store_true", help="add the batched-scenes comparison")
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--closure", action="store_true", help="add the learned-closure comparison")
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--closure-steps", type=int, default=1000)
    ap.add_argument("--search", action="store_true", help="add the list-based neighbour-search comparison")
    ap.add_argument("--search-steps", type=int, default=100)
    ap.add_argument("--search-mode", type=int, default=0, help="neighbour search of --plain-steps (0, 1, 2)")
    ap.add_argument("--voxel", action="store_true", help="add the voxel-density comparison")
    ap.add_argument("--obstacles", action="store_true", help="add the obstacle-avoidance comparison")
    ap.add_argument("--voxel-plain", action="store_true", help="--plain-steps with the voxel field on")
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (calibrates the HBM "
                         "byte counters of a profiler against a kernel of known traffic) and exit")
    ap.add_argument("--plain-steps", type=int, default=0, metavar="N",
                    help="only run N plain steps of the workload (no events, no graph) and exit: the command "
                         "for profiler counter passes")
    ap.add_argument("--tuning", default="", metavar="FUSED,VARIANT,TILE_X",
                    help="execution form for --plain-steps (default: the library's)")
    args = ap.parse_args()
    if args.copy_kernel:
        import torch

        nbytes = args.copy_kernel << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel_bytes_read": nbytes, "copy_kernel_bytes_written": nbytes, "launches": 5}))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the step is single-device).",
              file=sys.stderr)
        return 2

    import torch

    import paper_2311_15088_amd as sph
    from paper_2311_15088_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sc = scenes.config1()
    if args.plain_steps:
        sim = sph.create(sc)
        if args.tuning:
            sim.set_tuning(*[int(t) for t in args.tuning.split(",")])
        if args.search_mode:
            sim.set_search(args.search_mode)
        if args.voxel_plain:
            h = sc.params["h"]
            sim.enable_voxels(0.5 * h, h, 0.25 * h)
        sim.step(args.plain_steps)
        torch.cuda.synchronize()
        log(f"[bench] {args.plain_steps} plain steps done, tuning {sim.tuning()}")
        sim.close()
        return 0
    K, W = args.steps, args.warmup
    log(f"[bench] workload c1: n={sc.n} agents={sc.n_agents} steps={K} warmup={W}")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    inputs = [torch.from_numpy(a).to(dev) for a in (sc.x, sc.v, sc.y, sc.u)]
    torch.cuda.synchronize()

    def make():
        return sph.Simulation(sc.params, *inputs, stream=stream)

    # ---- timed region: K steps, HIP events at the density and force kernels ----
    sim = make()
    info = sim.info()
    sim.step_timed(W)
    torch.cuda.synchronize()
    pairs0 = int(sim.read(sph.PAIR_COUNT)[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms = sim.step_timed(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = int(sim.read(sph.PAIR_COUNT)[0]) - pairs0
    sim.close()
    ms_per_step = 1e3 * wall / K
    log(f"[bench] timed region: {ms_per_step:.4f} ms/step wall; density {1e3 * kernel_ms['density'] / K:.2f} us, "
        f"force_integrate {1e3 * kernel_ms['force_integrate'] / K:.2f} us per step")

    # ---- phase region: same K steps, an event between every two phases ----
    sim = make()
    sim.step_profiled(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phase_ms = sim.step_profiled(K)
    torch.cuda.synchronize()
    phase_wall_ms = 1e3 * (time.perf_counter() - t0) / K
    sim.close()
    log(f"[bench] phase region: {phase_wall_ms:.4f} ms/step wall, {sum(phase_ms.values()) / K:.4f} ms/step in phases")
    for k, vms in phase_ms.items():
        log(f"[bench]   {k:16s} {1e3 * vms / K:9.2f} us/step")

    # ---- graph region: same K steps replayed from captured graphs ----
    graph_ms = None
    if not args.no_graph:
        sim = make()
        sim.step(W)
        c = max(1, min(args.chunk, K))
        sim.capture(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done + c <= K:
            sim.step(c)
            done += c
        if done < K:
            sim.capture(0)
            sim.step(K - done)
        torch.cuda.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t0) / K
        sim.close()
        log(f"[bench] graph region: {graph_ms:.4f} ms/step")

    n, cells, agents = sc.n, info["cells"], sc.n_agents
    value = K * n / wall
    # whole-step HBM fraction with B_alg = 154 + 24 C/N bytes per particle-step
    b_alg = 154.0 + 24.0 * cells / n
    hbm_frac_step = b_alg * n / (ms_per_step * 1e-3) / (PEAK_HBM_GBS * 1e9)
    # roofline of the dominant kernel (force + integration): bound by vector
    # ALU issue, not HBM (about 25 FP32 operations per byte it must move)
    dom = "force_integrate"
    t_dom = kernel_ms[dom] / K * 1e-3
    flop = (FLOP_FORCE_PER_PAIR * pairs / K + FLOP_FORCE_PER_PARTICLE * n)
    ach = flop / t_dom / 1e12
    ach_hbm = kernel_bytes(dom, n, cells, agents) / t_dom / 1e9
    result = {
        "metric": "particle-steps/s & %HBM roofline @1M SPH+boid; batched & surrogate vs plain",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dam break 128x64x128 = 1,048,576 particles + 1,024 boids, h=0.02, dt=2e-4",
                   "n": n, "agents": agents, "cells": cells},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_FP32_TFLOPS, "traffic": force_traffic(),
                     "traffic_unit": "bytes per launch", "traffic_measured_on": TRAFFIC_FORCE["measured_on"],
                     "flop_per_launch": flop, "us_per_launch": t_dom * 1e6,
                     "hbm_alg_GBs": ach_hbm, "hbm_alg_frac": ach_hbm / PEAK_HBM_GBS},
        "step_hbm_frac": hbm_frac_step,
        "b_alg_bytes_per_particle_step": b_alg,
        "pair_interactions_per_s": pairs / wall,
        "mean_neighbours": pairs / (K * n),
        "kernel_us_per_step": {k: 1e3 * vms / K for k, vms in kernel_ms.items()},
        "phase_region": {"ms_per_step": phase_wall_ms,
                         "us_per_step": {k: 1e3 * vms / K for k, vms in phase_ms.items()}},
        "graph_ms_per_step": graph_ms,
    }
    if args.scale:
        result["scale"] = scale_leg(sph, scenes, torch, args)
    if args.batched:
        result["batched"] = batched_leg(sph, scenes, torch, args)
    if args.closure:
        result["closure"] = closure_leg(sph, scenes, torch, args)
    if args.search:
        result["search"] = search_leg(sph, scenes, torch, args)
    if args.voxel:
        result["voxel"] = voxel_leg(sph, scenes, torch, args)
    if args.obstacles:
        result["obstacles"] = obstacle_leg(sph, scenes, torch, args)
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
