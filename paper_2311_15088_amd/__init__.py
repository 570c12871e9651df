"""MI355X-native SPH + boid time step -- Python binding of ``libsph.so``.

This module only marshals arguments for the C ABI declared in
``include/sph.h``; every step of the method runs in the library's HIP kernels.
Importing it does not need a GPU; creating a simulation does, and fails loudly
when ``libsph.so`` has not been built (``python -m paper_2311_15088_amd.build``).

Inputs may be numpy arrays (host) or torch tensors (host or device); torch is
used only for device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ENONFINITE, ESTATE, ENOTIMPL = 0, -1, -2, -3, -4, -5, -6, -7
FLAG_DIAGNOSTICS, FLAG_CHECK_FINITE, FLAG_FUSED, FLAG_FEATURES = 1, 2, 4, 8
CLOSURE_PARAMS, CLOSURE_FEATURES = 49795, 256
CLOSURE_STATE_FLOATS = 3 * CLOSURE_PARAMS + 2

# fields (sph_field)
POS, VEL, AGENT_POS, AGENT_VEL, DENSITY, NBR_COUNT, CELL_KEY, ACC_INT, ACC_COUPLE, TOUCHED, \
    AGENT_FORCE, AGENT_STEER, AGENT_COUNTS, SORTED_IDS, CELL_OFFSETS, AGENT_KEY, AGENT_SORTED_IDS, \
    AGENT_CELL_OFFSETS, PAIR_COUNT, AGENT_FEATURES, AGENT_FORCE_MODEL, NBR_LIST_COUNTS, NBR_LIST_OFFSETS, \
    NBR_LIST, VOXEL_FIELD = range(25)
# neighbour search of the fluid passes (sph_search_set)
SEARCH_TILES, SEARCH_SORTED_LIST, SEARCH_BUCKET_LIST = 0, 1, 2

_FIELD_DTYPE = {
    POS: (np.float32, 3), VEL: (np.float32, 3), AGENT_POS: (np.float32, 3), AGENT_VEL: (np.float32, 3),
    DENSITY: (np.float32, 1), NBR_COUNT: (np.uint32, 1), CELL_KEY: (np.uint32, 1), ACC_INT: (np.float32, 3),
    ACC_COUPLE: (np.float32, 3), TOUCHED: (np.uint32, 1), AGENT_FORCE: (np.float32, 3),
    AGENT_STEER: (np.float32, 3), AGENT_COUNTS: (np.uint32, 4), SORTED_IDS: (np.uint32, 1),
    CELL_OFFSETS: (np.uint32, 1), AGENT_KEY: (np.uint32, 1), AGENT_SORTED_IDS: (np.uint32, 1),
    AGENT_CELL_OFFSETS: (np.uint32, 1), PAIR_COUNT: (np.uint64, 1), AGENT_FEATURES: (np.uint16, 256),
    AGENT_FORCE_MODEL: (np.float32, 3), NBR_LIST_COUNTS: (np.uint32, 1), NBR_LIST_OFFSETS: (np.uint32, 1),
    NBR_LIST: (np.uint32, 1), VOXEL_FIELD: (np.float32, 1),
}


class SphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sph status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    """Mirror of ``sph_params``."""

    _fields_ = [
        ("h", ctypes.c_float), ("rest_density", ctypes.c_float), ("gas_k", ctypes.c_float),
        ("viscosity", ctypes.c_float), ("mass", ctypes.c_float), ("dt", ctypes.c_float),
        ("gravity", ctypes.c_float * 3), ("box_min", ctypes.c_float * 3), ("box_max", ctypes.c_float * 3),
        ("wall_restitution", ctypes.c_float),
        ("r_sep", ctypes.c_float), ("r_ali", ctypes.c_float), ("r_coh", ctypes.c_float),
        ("w_sep", ctypes.c_float), ("w_ali", ctypes.c_float), ("w_coh", ctypes.c_float),
        ("r_couple", ctypes.c_float), ("couple_factor", ctypes.c_float), ("v_min", ctypes.c_float),
        ("v_max", ctypes.c_float), ("n_buckets", ctypes.c_uint32), ("kernel_norm", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class Tuning(ctypes.Structure):
    """Mirror of ``sph_tuning``."""

    _fields_ = [("fused", ctypes.c_int32), ("variant", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("ms_per_step", ctypes.c_float)]

    def as_dict(self):
        return dict(fused=self.fused, variant=self.variant, tile_x=self.tile_x, ms_per_step=self.ms_per_step,
                    name=variant_name(self.fused, self.variant))


class TrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("val_fraction", ctypes.c_float), ("seed", ctypes.c_uint32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("train_loss", ctypes.c_float), ("val_rel_rms", ctypes.c_float), ("force_scale", ctypes.c_float),
                ("steps", ctypes.c_int32), ("seconds", ctypes.c_double)]


class ClosureStats(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("last_rel_rms", ctypes.c_float), ("checks", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("surrogate_steps", ctypes.c_int64), ("exact_steps", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_agents", ctypes.c_int64), ("dims", ctypes.c_int32 * 3),
        ("agent_dims", ctypes.c_int32 * 3), ("cells", ctypes.c_int64), ("agent_cells", ctypes.c_int64),
        ("cell", ctypes.c_float), ("agent_cell", ctypes.c_float), ("steps", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
    ]


EXPORTS = ("sph_create", "sph_create_batch", "sph_step", "sph_read", "sph_field_bytes", "sph_info_get",
           "sph_capture", "sph_abort_set", "sph_step_profiled", "sph_step_timed", "sph_phase_name", "sph_autotune", "sph_tuning_set",
           "sph_tuning_get", "sph_variant_count", "sph_variant_name", "sph_variant_tile_max", "sph_destroy", "sph_last_error",
           "sph_closure_create", "sph_closure_train", "sph_closure_predict", "sph_closure_predict_static", "sph_closure_gradient",
           "sph_closure_adam_step", "sph_closure_weights", "sph_closure_io", "sph_closure_destroy", "sph_closure_last_error",
           "sph_closure_attach", "sph_closure_stats_get")
STEP_PHASES = 8

_lib = None


def phase_name(p: int) -> str:
    """Name of kernel p of a step (0 <= p < STEP_PHASES)."""
    return lib().sph_phase_name(int(p)).decode()


def lib() -> ctypes.CDLL:
    """Load libsph.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_15088_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.sph_create.restype = ctypes.c_int
        L.sph_create.argtypes = [ctypes.POINTER(Params), i64, vp, vp, i64, vp, vp, vp, ctypes.POINTER(vp)]
        L.sph_create_batch.restype = ctypes.c_int
        L.sph_create_batch.argtypes = [ctypes.POINTER(Params), i32, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.sph_step.restype = ctypes.c_int
        L.sph_step.argtypes = [vp, i32]
        L.sph_read.restype = ctypes.c_int
        L.sph_read.argtypes = [vp, i32, vp, i64]
        L.sph_field_bytes.restype = i64
        L.sph_field_bytes.argtypes = [vp, i32]
        L.sph_info_get.restype = ctypes.c_int
        L.sph_info_get.argtypes = [vp, ctypes.POINTER(Info)]
        L.sph_abort_set.restype = ctypes.c_int
        L.sph_abort_set.argtypes = [vp, i32]
        L.sph_capture.restype = ctypes.c_int
        L.sph_capture.argtypes = [vp, i32]
        L.sph_step_profiled.restype = ctypes.c_int
        L.sph_step_profiled.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i32]
        L.sph_step_timed.restype = ctypes.c_int
        L.sph_step_timed.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.sph_phase_name.restype = ctypes.c_char_p
        L.sph_phase_name.argtypes = [i32]
        L.sph_autotune.restype = ctypes.c_int
        L.sph_autotune.argtypes = [vp, i32, ctypes.POINTER(Tuning)]
        L.sph_tuning_set.restype = ctypes.c_int
        L.sph_tuning_set.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.sph_tuning_get.restype = ctypes.c_int
        L.sph_tuning_get.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.sph_variant_count.restype = i32
        L.sph_variant_count.argtypes = [i32]
        L.sph_variant_tile_max.restype = i32
        L.sph_variant_tile_max.argtypes = [i32, i32]
        L.sph_voxel_enable.restype = ctypes.c_int
        L.sph_voxel_enable.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.POINTER(i32)]
        L.sph_obstacles_set.restype = ctypes.c_int
        L.sph_obstacles_set.argtypes = [vp, i32, vp, ctypes.c_float, ctypes.c_float]
        L.sph_search_set.restype = ctypes.c_int
        L.sph_search_set.argtypes = [vp, i32, i32, i32]
        L.sph_variant_name.restype = ctypes.c_char_p
        L.sph_variant_name.argtypes = [i32, i32]
        L.sph_closure_create.restype = ctypes.c_int
        L.sph_closure_create.argtypes = [vp, ctypes.c_float, vp, ctypes.POINTER(vp)]
        L.sph_closure_train.restype = ctypes.c_int
        L.sph_closure_train.argtypes = [vp, vp, vp, i64, ctypes.POINTER(TrainParams), ctypes.POINTER(TrainReport)]
        L.sph_closure_predict.restype = ctypes.c_int
        L.sph_closure_predict.argtypes = [vp, vp, i64, vp]
        L.sph_closure_predict_static.restype = ctypes.c_int
        L.sph_closure_predict_static.argtypes = [vp, vp, i64, vp]
        L.sph_closure_io.restype = ctypes.c_int
        L.sph_closure_io.argtypes = [vp, i32, vp, i64]
        L.sph_closure_gradient.restype = ctypes.c_int
        L.sph_closure_gradient.argtypes = [vp, vp, vp, i64, vp, vp]
        L.sph_closure_adam_step.restype = ctypes.c_int
        L.sph_closure_adam_step.argtypes = [vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float]
        L.sph_closure_weights.restype = ctypes.c_int
        L.sph_closure_weights.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_float)]
        L.sph_closure_destroy.restype = None
        L.sph_closure_destroy.argtypes = [vp]
        L.sph_closure_last_error.restype = ctypes.c_char_p
        L.sph_closure_last_error.argtypes = [vp]
        L.sph_closure_attach.restype = ctypes.c_int
        L.sph_closure_attach.argtypes = [vp, vp, i32, ctypes.c_float]
        L.sph_closure_stats_get.restype = ctypes.c_int
        L.sph_closure_stats_get.argtypes = [vp, ctypes.POINTER(ClosureStats)]
        L.sph_destroy.restype = None
        L.sph_destroy.argtypes = [vp]
        L.sph_last_error.restype = ctypes.c_char_p
        L.sph_last_error.argtypes = [vp]
        _lib = L
    return _lib


def variant_name(fused: int, variant: int) -> Optional[str]:
    n = lib().sph_variant_name(int(fused), int(variant))
    return n.decode() if n else None


def variant_count(fused: int) -> int:
    return int(lib().sph_variant_count(int(fused)))


def variant_tile_max(fused: int, variant: int) -> int:
    """Widest tile_x the variant accepts."""
    return int(lib().sph_variant_tile_max(int(fused), int(variant)))


def params(d: Dict, flags: int = 0) -> Params:
    """Build an ``sph_params`` from a dict with the same field names."""
    p = Params()
    for name, _ in Params._fields_:
        if name == "flags":
            continue
        val = d[name]
        if isinstance(val, (list, tuple, np.ndarray)):
            arr = getattr(p, name)
            for k in range(3):
                arr[k] = float(val[k])
        elif name in ("n_buckets", "kernel_norm"):
            setattr(p, name, int(val))
        else:
            setattr(p, name, float(val))
    p.flags = int(flags) | int(d.get("flags", 0))
    return p


def _ptr(a):
    """(pointer, keepalive) for a numpy array or torch tensor of float32 [n][3]."""
    if a is None:
        return None, None
    if hasattr(a, "data_ptr"):  # torch tensor (host or device)
        t = a.contiguous()
        return (t.data_ptr() if t.numel() else None), t
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return (arr.ctypes.data if arr.size else None), arr


def _check(status: int, ctx=None):
    if status != OK:
        msg = lib().sph_last_error(ctx).decode(errors="replace")
        raise SphError(status, msg)


class Simulation:
    """One context: a single scene (``Simulation(...)``) or many (``Simulation.batch(...)``)."""

    def __init__(self, p: Dict, x, v, y, u, stream: int = 0, flags: int = 0, _ctx=None):
        self._ctx = _ctx
        if _ctx is not None:
            return
        L = lib()
        n = int(x.shape[0])
        na = int(y.shape[0])
        px, kx = _ptr(x)
        pv, kv = _ptr(v)
        py, ky = _ptr(y)
        pu, ku = _ptr(u)
        out = ctypes.c_void_p()
        prm = params(p, flags)
        _check(L.sph_create(ctypes.byref(prm), n, px, pv, na, py, pu, ctypes.c_void_p(stream), ctypes.byref(out)))
        self._ctx = out

    @classmethod
    def batch(cls, per_scene: Sequence[Dict], xs, vs, ys, us, stream: int = 0, flags: int = 0) -> "Simulation":
        L = lib()
        S = len(per_scene)
        prm = (Params * S)(*[params(p, flags) for p in per_scene])
        poff = np.zeros(S + 1, np.int64)
        aoff = np.zeros(S + 1, np.int64)
        poff[1:] = np.cumsum([int(x.shape[0]) for x in xs])
        aoff[1:] = np.cumsum([int(y.shape[0]) for y in ys])
        cat = lambda arrs: np.ascontiguousarray(np.concatenate([np.asarray(a, np.float32).reshape(-1, 3) for a in arrs]))  # noqa: E731
        X, V, Y, U = cat(xs), cat(vs), cat(ys), cat(us)
        out = ctypes.c_void_p()
        _check(L.sph_create_batch(prm, S, poff.ctypes.data, aoff.ctypes.data, X.ctypes.data if X.size else None,
                                  V.ctypes.data if V.size else None, Y.ctypes.data if Y.size else None,
                                  U.ctypes.data if U.size else None, ctypes.c_void_p(stream), ctypes.byref(out)))
        sim = cls(None, None, None, None, None, _ctx=out)
        sim.part_off, sim.agent_off = poff, aoff
        return sim

    # -- calls ------------------------------------------------------------
    def step(self, n: int = 1) -> None:
        _check(lib().sph_step(self._ctx, int(n)), self._ctx)

    def set_abort(self, raise_flag: bool) -> None:
        """Raise or clear the fused step's sticky abort flag (sph_abort_set)."""
        _check(lib().sph_abort_set(self._ctx, int(bool(raise_flag))), self._ctx)

    def capture(self, n: int) -> None:
        _check(lib().sph_capture(self._ctx, int(n)), self._ctx)

    def step_profiled(self, n: int) -> Dict[str, float]:
        """Run n directly launched steps; summed ms per phase (density and force timed at the
        kernels' own start and end, the other phases by events between launches)."""
        buf = (ctypes.c_double * STEP_PHASES)()
        _check(lib().sph_step_profiled(self._ctx, int(n), buf, STEP_PHASES), self._ctx)
        return {lib().sph_phase_name(p).decode(): buf[p] for p in range(STEP_PHASES)}

    def step_timed(self, n: int) -> Dict[str, float]:
        """Run n directly launched steps with events only at the density and force kernels'
        start and end; summed ms of those two kernels."""
        buf = (ctypes.c_double * 2)()
        _check(lib().sph_step_timed(self._ctx, int(n), buf), self._ctx)
        return {"density": buf[0], "force_integrate": buf[1]}

    def autotune(self, steps_per_trial: int = 5) -> Dict:
        """Time every execution form on this state (restored afterwards); keep the fastest."""
        t = Tuning()
        _check(lib().sph_autotune(self._ctx, int(steps_per_trial), ctypes.byref(t)), self._ctx)
        return t.as_dict()

    def set_tuning(self, fused: int, variant: int, tile_x: int = 32) -> None:
        """Execution form: fused (0/1), kernel variant, cells per fluid tile along x."""
        t = Tuning(int(fused), int(variant), int(tile_x), 0.0)
        _check(lib().sph_tuning_set(self._ctx, ctypes.byref(t)), self._ctx)

    def set_search(self, mode: int, bucket_capacity: int = 0, list_per_particle: int = 0) -> None:
        """Neighbour search of the fluid passes: SEARCH_TILES, SEARCH_SORTED_LIST or SEARCH_BUCKET_LIST."""
        _check(lib().sph_search_set(self._ctx, int(mode), int(bucket_capacity), int(list_per_particle)), self._ctx)

    def set_obstacles(self, boxes, vertex_spacing: float, weight: float) -> None:
        """Axis-aligned obstacle boxes [n, 6] (min xyz, max xyz); an empty list removes them."""
        b = np.ascontiguousarray(np.asarray(boxes, np.float32).reshape(-1, 6))
        _check(lib().sph_obstacles_set(self._ctx, int(b.shape[0]), b.ctypes.data if b.size else None,
                                       float(vertex_spacing), float(weight)), self._ctx)

    def enable_voxels(self, spacing: float, radius: float, particle_radius: float):
        """Voxel density at cube corners from the next step on; returns the corners per axis (x, y, z).
        spacing <= 0 turns it off."""
        dims = (ctypes.c_int32 * 3)()
        _check(lib().sph_voxel_enable(self._ctx, float(spacing), float(radius), float(particle_radius), dims),
               self._ctx)
        self.voxel_dims = tuple(dims)
        return self.voxel_dims

    def tuning(self) -> Dict:
        t = Tuning()
        _check(lib().sph_tuning_get(self._ctx, ctypes.byref(t)), self._ctx)
        return t.as_dict()

    def attach_closure(self, closure: Optional["Closure"], check_every: int = 50, max_rel_rms: float = 0.02) -> None:
        self._closure = closure  # keeps the closure alive while attached
        _check(lib().sph_closure_attach(self._ctx, closure._cl if closure else None, int(check_every),
                                        float(max_rel_rms)), self._ctx)

    def closure_stats(self) -> Dict:
        st = ClosureStats()
        _check(lib().sph_closure_stats_get(self._ctx, ctypes.byref(st)), self._ctx)
        return {k: getattr(st, k) for k, _ in ClosureStats._fields_}

    def field_bytes(self, field: int) -> int:
        b = lib().sph_field_bytes(self._ctx, int(field))
        if b < 0:
            _check(int(b), self._ctx)
        return int(b)

    def read(self, field: int) -> np.ndarray:
        """Copy a field to a new host numpy array (synchronises the stream)."""
        dt, w = _FIELD_DTYPE[field]
        nbytes = self.field_bytes(field)
        out = np.empty(nbytes // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().sph_read(self._ctx, int(field), out.ctypes.data if nbytes else None, nbytes), self._ctx)
        return out.reshape(-1, w) if w > 1 else out

    def read_into(self, field: int, tensor) -> None:
        """Enqueue a copy of a field into a (device) torch tensor."""
        nbytes = self.field_bytes(field)
        if tensor.numel() * tensor.element_size() < nbytes:
            raise ValueError("tensor too small")
        _check(lib().sph_read(self._ctx, int(field), ctypes.c_void_p(tensor.data_ptr()),
                              tensor.numel() * tensor.element_size()), self._ctx)

    def info(self) -> Dict:
        inf = Info()
        _check(lib().sph_info_get(self._ctx, ctypes.byref(inf)), self._ctx)
        return dict(n=inf.n, n_agents=inf.n_agents, dims=tuple(inf.dims), agent_dims=tuple(inf.agent_dims),
                    cells=inf.cells, agent_cells=inf.agent_cells, cell=inf.cell, agent_cell=inf.agent_cell,
                    steps=inf.steps, device_bytes=inf.device_bytes)

    def close(self) -> None:
        if self._ctx:
            lib().sph_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def create(scene, stream: int = 0, flags: int = 0) -> Simulation:
    """Simulation of a ``scenes.Scene``."""
    return Simulation(scene.params, scene.x, scene.v, scene.y, scene.u, stream=stream, flags=flags)


def create_batch(scene_list, stream: int = 0, flags: int = 0) -> Simulation:
    return Simulation.batch([s.params for s in scene_list], [s.x for s in scene_list], [s.v for s in scene_list],
                            [s.y for s in scene_list], [s.u for s in scene_list], stream=stream, flags=flags)


def _cl_check(status: int, cl=None):
    if status != OK:
        msg = lib().sph_closure_last_error(cl).decode(errors="replace")
        raise SphError(status, msg)


def _dptr(t):
    """Device pointer of a torch tensor (must be contiguous)."""
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Closure:
    """The learned coupling closure (weights, Adam state) on the device."""

    def __init__(self, weights=None, force_scale: float = 1.0, stream: int = 0):
        self._cl = ctypes.c_void_p()
        keep = None
        ptr = None
        if weights is not None:
            if hasattr(weights, "data_ptr"):
                keep = weights.contiguous()
                ptr = keep.data_ptr()
            else:
                keep = np.ascontiguousarray(np.asarray(weights, np.float32).ravel())
                if keep.size != CLOSURE_PARAMS:
                    raise ValueError(f"need {CLOSURE_PARAMS} weights")
                ptr = keep.ctypes.data
        _cl_check(lib().sph_closure_create(ptr, float(force_scale), ctypes.c_void_p(stream), ctypes.byref(self._cl)))

    def train(self, features, forces, epochs=20, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              val_fraction=0.1, seed=0) -> Dict:
        """features: device tensor [n, 256] of bfloat16 bits; forces: device float32 [n, 3]."""
        tp = TrainParams(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                         float(val_fraction), int(seed))
        rep = TrainReport()
        _cl_check(lib().sph_closure_train(self._cl, _dptr(features), _dptr(forces), int(features.shape[0]),
                                          ctypes.byref(tp), ctypes.byref(rep)), self._cl)
        return {k: getattr(rep, k) for k, _ in TrainReport._fields_}

    def predict(self, features, out):
        _cl_check(lib().sph_closure_predict(self._cl, _dptr(features), int(features.shape[0]), _dptr(out)), self._cl)
        return out

    def predict_static(self, features, out):
        """predict() without allocating: activations in the library's fixed device array
        (at most 65,536 rows per call)."""
        _cl_check(lib().sph_closure_predict_static(self._cl, _dptr(features), int(features.shape[0]), _dptr(out)),
                  self._cl)
        return out

    def save_state(self) -> np.ndarray:
        """Weights, Adam moments, force scale and Adam step count (sph_closure_io)."""
        buf = np.zeros(CLOSURE_STATE_FLOATS, np.float32)
        _cl_check(lib().sph_closure_io(self._cl, 0, buf.ctypes.data, buf.nbytes), self._cl)
        return buf

    def load_state(self, buf) -> None:
        b = np.ascontiguousarray(np.asarray(buf, np.float32))
        _cl_check(lib().sph_closure_io(self._cl, 1, b.ctypes.data, b.nbytes), self._cl)

    def gradient(self, features, forces):
        g = np.zeros(CLOSURE_PARAMS, np.float32)
        loss = ctypes.c_float()
        _cl_check(lib().sph_closure_gradient(self._cl, _dptr(features), _dptr(forces), int(features.shape[0]),
                                             g.ctypes.data, ctypes.addressof(loss)), self._cl)
        return g, loss.value

    def adam_step(self, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        g = np.ascontiguousarray(np.asarray(grad, np.float32))
        _cl_check(lib().sph_closure_adam_step(self._cl, g.ctypes.data, int(t), float(lr), float(beta1), float(beta2),
                                              float(eps)), self._cl)

    def weights(self):
        w = np.zeros(CLOSURE_PARAMS, np.float32)
        sc = ctypes.c_float()
        _cl_check(lib().sph_closure_weights(self._cl, 0, w.ctypes.data, ctypes.byref(sc)), self._cl)
        return w, sc.value

    def set_weights(self, w=None, force_scale=None):
        arr = None if w is None else np.ascontiguousarray(np.asarray(w, np.float32))
        sc = None if force_scale is None else ctypes.c_float(float(force_scale))
        _cl_check(lib().sph_closure_weights(self._cl, 1, None if arr is None else arr.ctypes.data,
                                            None if sc is None else ctypes.byref(sc)), self._cl)

    def close(self):
        if self._cl:
            lib().sph_closure_destroy(self._cl)
            self._cl = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
