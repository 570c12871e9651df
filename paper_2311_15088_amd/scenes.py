"""Seeded synthetic inputs for the SPH + boid time step.

This module only *generates inputs*: lattice sites, jitter, agent placement and
the scalar parameters of each workload.  It holds none of the time step's
arithmetic (no kernels, neighbour tests, forces or integration), so the HIP
path and the CPU reference draw identical inputs from it without sharing any
of the method.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw ``k`` of stream ``s`` under seed ``S`` is
``splitmix64(S * 2**32 + s * 2**40 + k)``, mapped to a double in [0, 1) from
its top 53 bits.  Every value is computed in float64 and rounded once to
float32.

Workloads follow the paper's setting: a block of fluid particles released in
the corner of a box (a dam break) under gravity, with boid agents placed in
the box (Sections "Underwater Agent Behaviors" and "Boid Motion and Agent
Fluid Interaction"), the smoothing length ``h``, rest density, gas constant
and viscosity of Section "Pressure and Viscosity", and the particle mass
``m = rest_density * s**3`` of a lattice of spacing ``s = h/2``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np

SEED0 = 0x23115088

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to ``counter + golden gamma`` (uint64 wraps)."""
    with np.errstate(over="ignore"):
        z = counter.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Counter-based uniform doubles in [0, 1) for draw indices ``idx``."""
    base = np.uint64((int(seed) * (1 << 32) + int(stream) * (1 << 40)) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        z = splitmix64(np.asarray(idx, dtype=np.uint64) + base)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform(seed: int, stream: int, n: int, lo, hi) -> np.ndarray:
    """``n`` x 3 uniform points in the box [lo, hi] (float64)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    u = uniform01(seed, stream, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    return lo + u * (hi - lo)


def unit_dirs(seed: int, stream: int, n: int) -> np.ndarray:
    """Isotropic unit vectors: z = 2u1 - 1, phi = 2 pi u2."""
    u = uniform01(seed, stream, np.arange(2 * n, dtype=np.uint64)).reshape(n, 2)
    z = 2.0 * u[:, 0] - 1.0
    phi = 2.0 * math.pi * u[:, 1]
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def gaussian(seed: int, stream: int, n: int) -> np.ndarray:
    """``n`` x 3 standard normal draws by Box-Muller."""
    u = uniform01(seed, stream, np.arange(6 * n, dtype=np.uint64)).reshape(n, 3, 2)
    u1 = 1.0 - u[..., 0]  # (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u[..., 1])


def lattice(nx: int, ny: int, nz: int, s: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Sites ``origin + (i + 0.5) s`` with x varying fastest, then y, then z."""
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    iz = np.arange(nz, dtype=np.float64)
    z, y, x = np.meshgrid(iz, iy, ix, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return np.asarray(origin, dtype=np.float64) + (pts + 0.5) * s


@dataclasses.dataclass
class Scene:
    """One workload: parameters plus float32 state in creation-id order."""

    name: str
    params: Dict
    x: np.ndarray  # [n, 3] fluid positions
    v: np.ndarray  # [n, 3] fluid velocities
    y: np.ndarray  # [a, 3] agent positions
    u: np.ndarray  # [a, 3] agent velocities
    steps: int

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_agents(self) -> int:
        return int(self.y.shape[0])


def default_params(h: float, dt: float, box_min, box_max, spacing: float | None = None) -> Dict:
    """Parameter set shared by every workload (reading of the paper's constants).

    rest density 1000, gas constant 3 (p = 3 (rho - 1000)), viscosity 0.1,
    mass rest_density * s^3 with s = h/2, gravity -9.81 along z, boid radii
    2h / 4h / 4h with weights 1.5 / 1 / 1, coupling radius 2h, speed limits
    [0.25, 1.0], wall restitution 0.5.
    """
    s = 0.5 * h if spacing is None else spacing
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    return dict(
        h=f32(h), rest_density=1000.0, gas_k=3.0, viscosity=f32(0.1), mass=f32(1000.0 * s ** 3),
        dt=f32(dt), gravity=[0.0, 0.0, f32(-9.81)],
        box_min=[f32(c) for c in box_min], box_max=[f32(c) for c in box_max],
        wall_restitution=0.5,
        r_sep=f32(2 * h), r_ali=f32(4 * h), r_coh=f32(4 * h), w_sep=1.5, w_ali=1.0, w_coh=1.0,
        r_couple=f32(2 * h), couple_factor=1.0, v_min=0.25, v_max=1.0,
        n_buckets=0, kernel_norm=0,
    )


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _jitter(pts: np.ndarray, amp: float, seed: int, stream: int) -> np.ndarray:
    u = uniform01(seed, stream, np.arange(pts.size, dtype=np.uint64)).reshape(pts.shape)
    return pts + (2.0 * u - 1.0) * amp


def dam_break(name: str, nx: int, ny: int, nz: int, h: float, box_min, box_max, n_agents: int,
              dt: float, steps: int, seed: int, agents: str = "above", n_truncate: int | None = None,
              spacing: float | None = None) -> Scene:
    """A jittered lattice block in the box corner plus agents.

    agents: "above" (uniform over the box above the fluid top + 2h),
            "upper" (uniform in the upper half of the box),
            "inside" (uniform in the fluid block's interior bounding box).
    """
    s = 0.5 * h if spacing is None else spacing
    bmin = np.asarray(box_min, dtype=np.float64)
    bmax = np.asarray(box_max, dtype=np.float64)
    pts = lattice(nx, ny, nz, s, bmin)
    if n_truncate is not None:
        pts = pts[:n_truncate]
    pts = _jitter(pts, 0.05 * h, seed, 0)
    n = pts.shape[0]
    top = bmin[2] + nz * s
    eps = 0.25 * h
    if agents == "above":
        lo = np.array([bmin[0] + eps, bmin[1] + eps, min(top + 2 * h, bmax[2] - 2 * eps)])
        hi = bmax - eps
    elif agents == "upper":
        lo = np.array([bmin[0] + eps, bmin[1] + eps, 0.5 * (bmin[2] + bmax[2])])
        hi = bmax - eps
    elif agents == "inside":
        lo = bmin + s + h
        hi = bmin + np.array([nx, ny, nz]) * s - h
    else:
        raise ValueError(agents)
    y = uniform(seed, 1, n_agents, lo, hi)
    u = 0.5 * unit_dirs(seed, 2, n_agents)
    return Scene(name=name, params=default_params(h, dt, bmin, bmax, s), x=_f32(pts),
                 v=np.zeros((n, 3), np.float32), y=_f32(y), u=_f32(u), steps=steps)


def config0(agents: str = "upper") -> Scene:
    """4,096 particles (16^3 lattice, s = h/2, h = 0.05) in [0,1]^3; 16 agents; dt 5e-4; 10 steps."""
    return dam_break("c0" if agents == "upper" else "c0c", 16, 16, 16, 0.05, (0, 0, 0), (1, 1, 1), 16,
                     5e-4, 10, SEED0 + 0x000, agents=agents)


def config0c() -> Scene:
    """Config 0 with the 16 agents inside the fluid, so that coupling is exercised."""
    return config0(agents="inside")


def config1() -> Scene:
    """1,048,576 particles: 128x64x128 column, s = 0.01, h = 0.02, box [0,3]x[0,1]x[0,3]; 1,024 agents above."""
    return dam_break("c1", 128, 64, 128, 0.02, (0, 0, 0), (3, 1, 3), 1024, 2e-4, 1000, SEED0 + 0x100)


def config4(agents: str = "inside") -> Scene:
    """4,194,304 particles: 256x64x256 column as config 1; 65,536 agents in the column's bounding box."""
    return dam_break("c4", 256, 64, 256, 0.02, (0, 0, 0), (3, 1, 3), 65536, 2e-4, 1000, SEED0 + 0x400,
                     agents=agents)


def config2() -> Scene:
    """16,777,216 particles in two blocks of unequal height; h = 0.01; 2^24 cells; 65,536 agents in 64 flocks."""
    seed = SEED0 + 0x200
    h, s = 0.01, 0.005
    a = lattice(128, 256, 384, s, (0.0, 0.0, 0.0))
    b = lattice(128, 256, 128, s, (1.92, 0.0, 0.0))
    pts = _jitter(np.concatenate([a, b]), 0.05 * h, seed, 0)
    del a, b
    sigma = 8 * h
    centres = uniform(seed, 3, 64, [3 * sigma] * 3, [2.56 - 3 * sigma] * 3)
    y = np.repeat(centres, 1024, axis=0) + sigma * gaussian(seed, 4, 65536)
    y = np.clip(y, 0.25 * h, 2.56 - 0.25 * h)
    u = 0.5 * unit_dirs(seed, 2, 65536)
    p = default_params(h, 1e-4, (0, 0, 0), (2.56, 2.56, 2.56), s)
    p["n_buckets"] = 1 << 24
    n = pts.shape[0]
    return Scene("c2", p, _f32(pts), np.zeros((n, 3), np.float32), _f32(y), _f32(u), 200)


def batched_specs(n_scenes: int = 512, seed: int = SEED0 + 0x300,
                  n_range=(2048, 262144), a_range=(4, 512), h_range=(0.01, 0.05)) -> List[Dict]:
    """Per-scene sizes of the batched workload (log-uniform N, uniform A, h, aspect)."""
    u = uniform01(seed, 5, np.arange(4 * n_scenes, dtype=np.uint64)).reshape(n_scenes, 4)
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    specs = []
    for k in range(n_scenes):
        n = int(round(math.exp(lo + u[k, 0] * (hi - lo))))
        a = int(a_range[0] + math.floor(u[k, 1] * (a_range[1] - a_range[0] + 1)))
        h = float(h_range[0] + u[k, 2] * (h_range[1] - h_range[0]))
        aspect = 0.5 + 1.5 * u[k, 3]
        specs.append(dict(n=n, a=min(a, a_range[1]), h=h, aspect=aspect))
    return specs


def batched_scene(spec: Dict, k: int, seed: int = SEED0 + 0x300, dt: float = 2e-4, steps: int = 100) -> Scene:
    """One dam-break scene of the batched workload: n_y = round(n_x/2), n_z = round(aspect n_x)."""
    n = spec["n"]
    nx = 1
    while True:
        ny = max(1, int(round(nx / 2)))
        nz = max(1, int(round(spec["aspect"] * nx)))
        if nx * ny * nz >= n:
            break
        nx += 1
    h = spec["h"]
    s = 0.5 * h
    box_max = (2.34 * nx * s, 1.56 * ny * s, 2.34 * nz * s)
    return dam_break(f"b{k}", nx, ny, nz, h, (0, 0, 0), box_max, spec["a"], dt, steps,
                     seed + 0x1000 + k, n_truncate=n)


def batched(n_scenes: int = 512, **kw) -> List[Scene]:
    """The batched workload: ``n_scenes`` independent dam breaks of uneven size."""
    return [batched_scene(sp, k) for k, sp in enumerate(batched_specs(n_scenes, **kw))]


def small_dam(nx=12, ny=10, nz=14, h=0.05, n_agents=24, agents="inside", seed=SEED0 + 0x777,
              box_max=(1.0, 0.8, 1.0), dt=5e-4) -> Scene:
    """A small ragged dam break (several cells and rows, uneven counts) for quick parity cases."""
    return dam_break("small", nx, ny, nz, h, (0, 0, 0), box_max, n_agents, dt, 5, seed, agents=agents)


def wall_scene():
    """Particles and agents placed just inside each wall, edge and corner of
    the unit box, moving outward fast enough that one step (dt = 5e-4, h =
    0.05) carries them through the wall, or, for a second set, not quite to
    it.  Returns (params, x, v, y, u, dt)."""
    p = default_params(0.05, 5e-4, (0, 0, 0), (1, 1, 1))
    dt = p["dt"]
    pts, vel = [], []
    # one particle per wall, crossing by 3e-4 (speed 1 over dt = 5e-4 from 2e-4 inside)
    # and a partner 3h away that stops 3e-4 short of the wall
    for axis in range(3):
        for side in (0, 1):
            for inset, tag in ((2e-4, "cross"), (8e-4, "short")):
                x = np.full(3, 0.5)
                x[(axis + 1) % 3] = 0.3 if tag == "cross" else 0.7
                x[axis] = inset if side == 0 else 1.0 - inset
                v = np.zeros(3)
                v[axis] = (-1.0 if side == 0 else 1.0)
                pts.append(x)
                vel.append(v)
    # corners and edges: crossing two and three walls at once
    for c in ((0, 0, 0), (1, 1, 1), (0, 1, 0), (1, 0, 1), (0, 0, 1)):
        c = np.asarray(c, np.float64)
        x = np.where(c == 0, 2e-4, 1.0 - 2e-4)
        v = np.where(c == 0, -1.0, 1.0)
        pts.append(x)
        vel.append(v)
    for e in ((0, 0, 0.5), (1, 0.5, 1)):
        e = np.asarray(e, np.float64)
        x = np.where(e == 0, 3e-4, np.where(e == 1, 1.0 - 3e-4, 0.5))
        v = np.where(e == 0, -1.0, np.where(e == 1, 1.0, 0.0))
        pts.append(x)
        vel.append(v)
    # a particle on the wall, moving out, and one on the wall moving in
    pts += [np.array([0.0, 0.2, 0.2]), np.array([1.0, 0.8, 0.8])]
    vel += [np.array([-0.5, 0.0, 0.0]), np.array([-0.5, 0.0, 0.0])]
    x = np.asarray(pts, np.float32)
    v = np.asarray(vel, np.float32)
    # agents: at top speed (v_max) through the walls
    ya = np.array([[3e-4, 0.5, 0.5], [0.5, 1 - 3e-4, 0.5], [0.5, 0.5, 3e-4], [1 - 1e-4, 1e-4, 1 - 1e-4]], np.float32)
    ua = np.array([[-1, 0, 0], [0, 1, 0], [0, 0, -1], [0.577, -0.577, 0.577]], np.float32)
    return p, x, v, ya, ua, dt


def clumped_dam(n_clump: int = 1500, side_cells: float = 2.0, seed: int = SEED0 + 0x778) -> Scene:
    """small_dam plus a dense clump: n_clump extra particles uniform in a cube of
    side_cells grid cells inside the fluid (a compressed region: cells far above
    the rest occupancy, neighbour counts in the hundreds)."""
    base = small_dam(seed=seed)
    h = base.params["h"]
    side = side_cells * h
    centre = np.array([0.3, 0.2, 0.25])
    extra = centre + uniform(seed, 3, n_clump, -0.5, 0.5) * side
    x = _f32(np.concatenate([base.x.astype(np.float64), extra]))
    v = np.zeros_like(x)
    return Scene("clumped", base.params, x, v, base.y, base.u, base.steps)


CONFIGS = {"c0": config0, "c0c": config0c, "c1": config1, "c2": config2, "c4": config4}


MLP_SIZES = (256, 128, 128, 3)


def mlp_init(seed: int = SEED0 + 0x500) -> Dict[str, np.ndarray]:
    """Initial closure weights: Kaiming-uniform U(-b, b), b = sqrt(6 / fan_in), zero biases.

    Weights are [fan_in, fan_out] float32; the flat parameter order is
    W1, b1, W2, b2, W3, b3 (49,795 values).
    """
    p = {}
    for layer in range(3):
        fi, fo = MLP_SIZES[layer], MLP_SIZES[layer + 1]
        b = math.sqrt(6.0 / fi)
        u = uniform01(seed, 10 + layer, np.arange(fi * fo, dtype=np.uint64)).reshape(fi, fo)
        p[f"W{layer + 1}"] = ((2.0 * u - 1.0) * b).astype(np.float32)
        p[f"b{layer + 1}"] = np.zeros(fo, np.float32)
    return p


def mlp_flat(p: Dict[str, np.ndarray]) -> np.ndarray:
    """Parameters in the flat order W1, b1, W2, b2, W3, b3 (float32)."""
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def mlp_unflat(flat: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for layer in range(3):
        fi, fo = MLP_SIZES[layer], MLP_SIZES[layer + 1]
        out[f"W{layer + 1}"] = np.asarray(flat[o:o + fi * fo]).reshape(fi, fo)
        o += fi * fo
        out[f"b{layer + 1}"] = np.asarray(flat[o:o + fo])
        o += fo
    return out
