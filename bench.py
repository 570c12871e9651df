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
    kernel durations of the roofline come from this region; its step time is
    reported as ms_per_step_direct_launches);
  * phase region: the same K steps with an event between every two phases
    as well (the per-phase breakdown; the extra events cost some time
    between launches, so its step time is reported but not used);
  * graph region: K steps replayed from captured HIP graphs, without events:
    the step time and `value` (with --no-graph, the timed region's).

`roofline` is that of the longer fluid pass of the timed region: its
algorithmic bytes per launch (18 B per particle for density, 52 B for force +
integration) over its average launch time, against 8 TB/s.  The force pass's
figures against the FP32 vector ALU, which is what bounds it, are under `alu`.

Then, unless left out: the 16.7M-particle scale workload (`scale`), 512
batched scenes against plain per-scene loops (`batched`), the learned coupling
closure against the exact gather on 4,194,304 particles and 65,536 agents
(`closure`), and the CPU oracle on the host cores (`cpu_baseline`).

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
ATTAINABLE_FP32_TFLOPS = 78.6
# dense bf16 MFMA peak of MI355X (without structured sparsity), TFLOP/s
PEAK_BF16_TFLOPS = 2500.0

# Algorithmic FP32 operations of the force + integration pass: per neighbour
# pair (i, j in N_i) the pair term of the pressure and viscosity forces
# (displacement 3, r^2 5, cut-off test 1, r, q, w 3, pressure coefficient 5,
# velocity difference and viscosity coefficient 4, pair vector 13, sum 3), and
# per particle the division by rho, coupling scale, gravity, Euler-Cromer
# update and walls.
FLOP_FORCE_PER_PAIR = 37
FLOP_FORCE_PER_PARTICLE = 30

# Algorithmic bytes per particle of the two fluid passes, each array counted
# once per pass: density reads x (12) and writes rho (4) and the neighbour
# count as 16 bits (2); force + integration reads x, v, rho (28) and writes
# x', v' (24).
B_ALG_PASS = {"density": 18, "force_integrate": 52}

# HBM traffic per launch of the fluid passes from two rocprofv3 counter runs
# (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads for a
# plain device copy of known size), averaged over the timed steps of the run
# named; valid only for the kernel sources it was measured on.
TRAFFIC = {
    "density": {"sources_sha256_16": "af7bd13abb1d2cc7", "bytes_per_launch": 106.6e6,
                "run": "bench.py --plain-steps 1025, dispatches 26-1025 (profiles/fluid_counters_dam_break_1M.md)"},
    "force_integrate": {"sources_sha256_16": "af7bd13abb1d2cc7", "bytes_per_launch": 196.2e6,
                        "run": "bench.py --plain-steps 1025, dispatches 26-1025 (profiles/fluid_counters_dam_break_1M.md)"},
}
FLUID_SOURCES = ("paper_2311_15088_amd/csrc/sph_fluid_impl.hpp", "paper_2311_15088_amd/csrc/sph_physics.hip",
                 "paper_2311_15088_amd/csrc/sph_internal.hpp", "paper_2311_15088_amd/csrc/sph_device.hpp")


def sources_hash():
    """Hash of the fluid kernels' code: the sources with their // comments and
    blank lines taken out, so that a comment edit keeps the measured traffic."""
    import hashlib

    h = hashlib.sha256()
    for f in FLUID_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    t = TRAFFIC.get(kernel)
    return t if t and t["sources_sha256_16"] == sources_hash() else None


# Algorithmic bytes per element and launch for each kernel of a step (the
# arrays each kernel must read and write once, in the layout it uses).
#   key_count      reads x,y,z (12), writes key, rank (8)             per particle
#   scan_reduce    reads cnt (4)                                       per cell
#   scan_apply     reads cnt (4), writes off (4), clears cnt (4)       per cell
#   scatter        reads key, rank, id (12), writes src, id (8)        per particle
#   fixup_tile_list reads src, id, key (12), x, v (24), writes x, v, id (28) per particle
#                  (the work-item list in the same launch: 8 per tile)
#   density        reads x (12), writes rho (4), n (2)                 per particle
#   force_integrate reads x, v, rho (28), writes x', v' (24)           per particle
#   agents         reads y, u (24), writes y', u' (24)                 per agent
B_PER_PARTICLE = {"key_count": 20, "scatter": 20, "fixup_tile_list": 64, "density": 18, "force_integrate": 52}
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


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy of `mib` MiB, timed with events: read + write bytes per second."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _oracle_rate(oracle, sc, budget_s, nbr_mode=1, max_steps=200):
    """Whole oracle steps of a scene from its initial state until budget_s."""
    x, v, y, u = sc.x, sc.v, sc.y, sc.u
    steps = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.step(sc.params, x, v, y, u, nbr_mode=nbr_mode)
        x, v = r["x1"].astype(np.float32), r["v1"].astype(np.float32)
        y, u = r["y1"].astype(np.float32), r["u1"].astype(np.float32)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= max_steps:
            return steps, el


def cpu_baseline(sc, budget_s: float, full: bool):
    """The CPU oracle timed on the host cores on whole steps of the same workload."""
    import oracle  # test infrastructure: only this leg of the bench uses it
    from paper_2311_15088_amd import scenes

    threads = oracle.threads()
    steps, el = _oracle_rate(oracle, sc, budget_s)
    out = {
        "value": steps * sc.n / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
        "sample": f"{steps} whole step(s) of the same {sc.n}-particle workload from its initial state, FP64 "
                  f"oracle with its cell-list neighbour finder (sets identical to brute force), "
                  f"{threads} OpenMP threads on '{cpu_model()}' (nproc {os.cpu_count()}), {el:.1f} s",
    }
    if full:
        # the same on one core
        oracle.set_threads(1)
        s1, e1 = _oracle_rate(oracle, sc, 0.5 * budget_s)
        out["one_core"] = {"value": s1 * sc.n / e1, "unit": "particle-steps/s", "cores": 1,
                           "sample": f"{s1} whole step(s), {e1:.1f} s"}
        oracle.set_threads(threads)
        # brute force (the oracle's definition): config 0 for its 10 steps ...
        c0 = scenes.config0()
        s0, e0 = _oracle_rate(oracle, c0, 1e9, nbr_mode=0, max_steps=10)
        out["brute_force_config0"] = {"value": s0 * c0.n / e0, "unit": "particle-steps/s", "cores": threads,
                                      "sample": f"{s0} whole steps of the 4,096-particle scene, {e0:.2f} s"}
        # ... and config 1 for one step on a sample of particles (every sampled
        # particle and every neighbour whose density it needs is tested against
        # all N particles)
        rng = np.random.default_rng(5)
        fs = np.sort(rng.choice(sc.n, 64, replace=False))
        t0 = time.perf_counter()
        r = oracle.step(sc.params, sc.x, sc.v, sc.y, sc.u, fsample=fs, asample=np.zeros(0, np.int64), nbr_mode=0)
        eb = time.perf_counter() - t0
        tested = int(len(fs) + r["nbr"][fs].sum())  # particles brute-forced (sample + density neighbours)
        out["brute_force_config1"] = {
            "particles_tested_per_s": tested / eb, "cores": threads,
            "full_step_s_estimate": eb * sc.n / tested,
            "sample": f"one step of 64 sampled particles of the same workload: {tested} particles tested "
                      f"against all {sc.n} in {eb:.2f} s"}
    return out


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
    """512 independent dam breaks of uneven size: one batched context (autotuned
    form, K steps in one graph) against a loop over the scenes with one plain
    context each, replayed from each scene's own graph of K steps, and against
    the same loop launched eagerly."""
    scs = scenes.batched(args.scenes)
    n_tot = sum(s.n for s in scs)
    log(f"[bench] batched: {len(scs)} scenes, {n_tot} particles, {sum(s.n_agents for s in scs)} agents")
    stream = torch.cuda.current_stream().cuda_stream
    K = args.batched_steps
    bat = sph.create_batch(scs, stream=stream)
    t0 = time.perf_counter()
    tuned = bat.autotune(2)
    t_tune = time.perf_counter() - t0
    log(f"[bench] batched autotune ({t_tune:.1f} s): {tuned}")

    def time_graph(sim):
        sim.step(2)
        sim.capture(K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(K)  # one graph of K steps
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    tb = time_graph(bat)
    # the persistent fused launch in its fastest variant, for the record
    fused = {}
    for v in range(sph.variant_count(1)):
        bat.set_tuning(1, v, tuned["tile_x"])
        fused[sph.variant_name(1, v)] = len(scs) * K / time_graph(bat)
    bat.close()
    # a loop of plain contexts, one per scene
    sims = [sph.create(sc, stream=stream) for sc in scs]
    for sim in sims:
        sim.step(2)
        sim.capture(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(K)  # each scene's own graph
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    for sim in sims:
        sim.capture(0)
    Ke = max(1, K // 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(Ke)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    rate = len(scs) * K / tb
    out = {
        "workload": f"{len(scs)} dam breaks, {n_tot} particles in total, N log-uniform in [2048, 262144]",
        "scenes": len(scs), "particles": n_tot, "steps": K,
        "scene_steps_per_s": rate, "particle_steps_per_s": n_tot * K / tb,
        "autotuned": tuned, "autotune_s": t_tune, "fused_scene_steps_per_s": fused,
        "plain_graph_loop_scene_steps_per_s": len(scs) * K / tg,
        "plain_eager_loop_scene_steps_per_s": len(scs) * Ke / te, "plain_eager_loop_steps": Ke,
        "speedup_vs_plain_graph_loop": rate / (len(scs) * K / tg),
        "speedup_vs_plain_eager_loop": rate / (len(scs) * Ke / te),
    }
    log(f"[bench] batched: {rate:.0f} scene-steps/s; plain graphs {out['plain_graph_loop_scene_steps_per_s']:.0f}, "
        f"plain eager {out['plain_eager_loop_scene_steps_per_s']:.0f}")
    return out


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
    # MFMA roofline of the network's forward pass (bf16 MFMA GEMMs with fused
    # bias and GELU epilogues): 65,536 rows, as many as config 4 has agents
    rows = min(65536, got)
    xf = X[:rows].contiguous()
    out = torch.empty((rows, 3), dtype=torch.float32, device=dev)
    for _ in range(3):
        cl.predict(xf, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        cl.predict(xf, out)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    flop = 2.0 * (256 * 128 + 128 * 128 + 128 * 3) * rows
    mlp = {"rows": rows, "gflop": flop / 1e9, "us": us, "achieved_tflops": flop / (us * 1e-6) / 1e12,
           "peak_tflops": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "bound": "mfma"}
    mlp["frac"] = mlp["achieved_tflops"] / PEAK_BF16_TFLOPS
    log(f"[bench] closure: forward of {rows} rows in {us:.1f} us = {mlp['achieved_tflops']:.1f} TFLOP/s")
    del X, F, xf, out
    # evaluation run: the workload itself, exact gather vs closure
    sc = scenes.config4()
    K = args.closure_steps
    res = {"pairs": got, "collect_s": t_collect, "train": rep, "steps": K, "mlp_forward_roofline": mlp}
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
    ap.add_argument("--cpu-full", action="store_true",
                    help="add the one-core and brute-force timings of the CPU oracle")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="leave out the 16.7M-particle scale workload")
    ap.add_argument("--scale-steps", type=int, default=50)
    ap.add_argument("--no-batched", action="store_true", help="leave out the batched-scenes comparison")
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--no-closure", action="store_true", help="leave out the learned-closure comparison")
    ap.add_argument("--pairs", type=int, default=262_144)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--closure-steps", type=int, default=100)
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
    ap.add_argument("--plain-workload", default="c1", choices=("c1", "c2", "c3", "c4"),
                    help="workload of --plain-steps: c1 the 1M dam break, c2 the 16.7M two-block scene, "
                         "c3 the 512 batched scenes (autotuned first), c4 the 4.2M / 65,536-agent scene")
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
        if args.plain_workload == "c3":
            scs = scenes.batched(args.scenes)
            sim = sph.create_batch(scs)
            if not args.tuning:
                log(f"[bench] batched plain steps: {len(scs)} scenes, autotuned {sim.autotune(2)}")
        else:
            if args.plain_workload != "c1":
                sc = scenes.config2() if args.plain_workload == "c2" else scenes.config4()
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
    # the whole job's rate: K steps replayed from captured graphs (the form a
    # caller stepping repeatedly uses), else the directly launched region
    direct_ms = ms_per_step
    if graph_ms is not None:
        ms_per_step = graph_ms
    value = K * n / (ms_per_step * 1e-3 * K)
    # whole-step HBM fraction with B_alg = 154 + 24 C/N bytes per particle-step
    b_alg = 154.0 + 24.0 * cells / n
    hbm_frac_step = b_alg * n / (ms_per_step * 1e-3) / (PEAK_HBM_GBS * 1e9)
    # roofline of the dominant kernel of this run (the longer fluid pass):
    # its algorithmic bytes per launch over its average launch duration
    dom = max(("density", "force_integrate"), key=lambda k: kernel_ms[k])
    t_dom = kernel_ms[dom] / K * 1e-3
    bytes_dom = B_ALG_PASS[dom] * n
    ach = bytes_dom / t_dom / 1e9
    tr = measured_traffic(dom)
    # the force pass against the FP32 vector ALU, which is what bounds it
    t_f = kernel_ms["force_integrate"] / K * 1e-3
    flop = (FLOP_FORCE_PER_PAIR * pairs / K + FLOP_FORCE_PER_PARTICLE * n)
    result = {
        "metric": "particle-steps/s & %HBM roofline @1M SPH+boid; batched & surrogate vs plain",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "ms_per_step_direct_launches": direct_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dam break 128x64x128 = 1,048,576 particles + 1,024 boids, h=0.02, dt=2e-4",
                   "n": n, "agents": agents, "cells": cells},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": ach / PEAK_HBM_GBS, "traffic": None if tr is None else tr["bytes_per_launch"],
                     "traffic_unit": "bytes per launch", "traffic_measured_on": None if tr is None else tr["run"],
                     "bytes_per_particle": B_ALG_PASS[dom], "particles_per_launch": n,
                     "us_per_launch": t_dom * 1e6},
        "alu": {"kernel": "force_integrate", "flop_per_launch": flop, "us_per_launch": t_f * 1e6,
                "achieved_tflops": flop / t_f / 1e12, "peak_tflops": PEAK_FP32_TFLOPS,
                "frac_of_peak": flop / t_f / 1e12 / PEAK_FP32_TFLOPS,
                "frac_of_attainable": flop / t_f / 1e12 / ATTAINABLE_FP32_TFLOPS},
        "kernels_hbm_frac": {k: B_ALG_PASS[k] * n / (kernel_ms[k] / K * 1e-3) / (PEAK_HBM_GBS * 1e9)
                             for k in B_ALG_PASS},
        "step_hbm_frac": hbm_frac_step,
        "b_alg_bytes_per_particle_step": b_alg,
        "pair_interactions_per_s": pairs / (ms_per_step * 1e-3 * K),
        "mean_neighbours": pairs / (K * n),
        "kernel_us_per_step": {k: 1e3 * vms / K for k, vms in kernel_ms.items()},
        "phase_region": {"ms_per_step": phase_wall_ms,
                         "us_per_step": {k: 1e3 * vms / K for k, vms in phase_ms.items()}},
        "graph_ms_per_step": graph_ms,
        "copy_kernel_GBs": copy_bandwidth(torch),
    }
    if not args.no_scale:
        result["scale"] = scale_leg(sph, scenes, torch, args)
    if not args.no_batched:
        result["batched"] = batched_leg(sph, scenes, torch, args)
    if not args.no_closure:
        result["closure"] = closure_leg(sph, scenes, torch, args)
    if args.search:
        result["search"] = search_leg(sph, scenes, torch, args)
    if args.voxel:
        result["voxel"] = voxel_leg(sph, scenes, torch, args)
    if args.obstacles:
        result["obstacles"] = obstacle_leg(sph, scenes, torch, args)
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget, args.cpu_full)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
