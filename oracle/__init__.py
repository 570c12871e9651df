"""CPU reference (oracle) for the SPH + boid time step and the coupling MLP.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2311_15088_amd``) and never imports it.

``step`` wraps the plain C implementation in ``sph_oracle.c`` (FP64 physics,
FP32 neighbour predicates, brute-force neighbour sets by definition).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "libsph_oracle.so")

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/libsph_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double), ("rest_density", ctypes.c_double), ("gas_k", ctypes.c_double),
        ("viscosity", ctypes.c_double), ("mass", ctypes.c_double), ("dt", ctypes.c_double),
        ("gravity", ctypes.c_double * 3), ("box_min", ctypes.c_double * 3), ("box_max", ctypes.c_double * 3),
        ("wall_restitution", ctypes.c_double),
        ("r_sep", ctypes.c_double), ("r_ali", ctypes.c_double), ("r_coh", ctypes.c_double),
        ("w_sep", ctypes.c_double), ("w_ali", ctypes.c_double), ("w_coh", ctypes.c_double),
        ("r_couple", ctypes.c_double), ("couple_factor", ctypes.c_double), ("v_min", ctypes.c_double),
        ("v_max", ctypes.c_double), ("kernel_norm", ctypes.c_int32), ("nbr_mode", ctypes.c_int32),
    ]


_U32P = ctypes.POINTER(ctypes.c_uint32)
_F64P = ctypes.POINTER(ctypes.c_double)


class _Out(ctypes.Structure):
    _fields_ = [
        ("key", _U32P), ("nbr", _U32P), ("touched", _U32P),
        ("rho", _F64P), ("a_int", _F64P), ("a_coup", _F64P), ("x1", _F64P), ("v1", _F64P),
        ("cnt", _U32P), ("off", _U32P), ("sorted", _U32P),
        ("akey", _U32P), ("n_sep", _U32P), ("n_ali", _U32P), ("n_coh", _U32P), ("n_cpl", _U32P),
        ("steer", _F64P), ("force", _F64P), ("y1", _F64P), ("u1", _F64P),
        ("acnt", _U32P), ("aoff", _U32P), ("asorted", _U32P),
        ("x1f", _F64P), ("v1f", _F64P), ("y1f", _F64P), ("u1f", _F64P),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_grid.restype = ctypes.c_int64
        L.orc_grid.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_Out)]
        L.orc_step_ex.restype = ctypes.c_int
        L.orc_step_ex.argtypes = L.orc_step.argtypes[:-1] + [ctypes.c_void_p, ctypes.POINTER(_Out)]
        L.orc_step_rho.restype = ctypes.c_int
        L.orc_step_rho.argtypes = L.orc_step_ex.argtypes[:-1] + [ctypes.c_void_p, ctypes.POINTER(_Out)]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _params(p: Dict, nbr_mode: int) -> _Params:
    s = _Params()
    for name, _ in _Params._fields_:
        if name == "nbr_mode":
            continue
        val = p[name]
        if isinstance(val, (list, tuple, np.ndarray)):
            arr = getattr(s, name)
            for k in range(3):
                arr[k] = float(np.float32(val[k]))
        elif name == "kernel_norm":
            s.kernel_norm = int(val)
        else:
            setattr(s, name, float(np.float32(val)))
    s.nbr_mode = int(nbr_mode)
    return s


def grid(p: Dict, agent: bool = False):
    """(dims, cell size, inverse cell size, number of cells) of the fluid or agent grid."""
    dims = (ctypes.c_int32 * 3)()
    cell = ctypes.c_float()
    inv = ctypes.c_float()
    nc = lib().orc_grid(ctypes.byref(_params(p, 0)), int(agent), dims, ctypes.byref(cell), ctypes.byref(inv))
    if nc <= 0:
        raise ValueError("invalid grid parameters")
    return tuple(dims), cell.value, inv.value, int(nc)


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle on n OpenMP threads from now on."""
    lib().orc_set_threads(int(n))


def _c(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def step(p: Dict, x, v, y, u, fsample: Optional[np.ndarray] = None, asample: Optional[np.ndarray] = None,
         nbr_mode: int = 0, agent_acc: Optional[np.ndarray] = None,
         rho_in: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """One reference time step from the float32 state (id order).

    Returns a dict of numpy arrays: cell keys, counts, offsets, sorted ids,
    neighbour counts, density, internal / coupling acceleration, new fluid
    state, agent keys and order, agent neighbour counts, steering, coupling
    force and new agent state; ``x1f``, ``v1f``, ``y1f``, ``u1f`` are the new
    states before the walls act.  ``agent_acc`` ([na, 3], id order) is a further
    steering acceleration added to the boid rules (obstacle avoidance,
    ``oracle/obstacles.py``).  ``rho_in`` ([n], id order) replaces the
    computed density in every force term (``rho`` still returns the computed
    one).  Entries outside ``fsample`` / ``asample`` are
    NaN (or 0xFFFFFFFF for counts).
    """
    x = _c(x, np.float32).reshape(-1, 3)
    v = _c(v, np.float32).reshape(-1, 3)
    y = _c(y, np.float32).reshape(-1, 3)
    u = _c(u, np.float32).reshape(-1, 3)
    n, na = x.shape[0], y.shape[0]
    _, _, _, nc = grid(p, False)
    _, _, _, nac = grid(p, True)
    r = dict(
        key=np.zeros(n, np.uint32), nbr=np.zeros(n, np.uint32), touched=np.zeros(n, np.uint32),
        rho=np.zeros(n), a_int=np.zeros((n, 3)), a_coup=np.zeros((n, 3)), x1=np.zeros((n, 3)),
        v1=np.zeros((n, 3)), cnt=np.zeros(nc, np.uint32), off=np.zeros(nc + 1, np.uint32),
        sorted=np.zeros(n, np.uint32), akey=np.zeros(na, np.uint32), n_sep=np.zeros(na, np.uint32),
        n_ali=np.zeros(na, np.uint32), n_coh=np.zeros(na, np.uint32), n_cpl=np.zeros(na, np.uint32),
        steer=np.zeros((na, 3)), force=np.zeros((na, 3)), y1=np.zeros((na, 3)), u1=np.zeros((na, 3)),
        acnt=np.zeros(nac, np.uint32), aoff=np.zeros(nac + 1, np.uint32), asorted=np.zeros(na, np.uint32),
        x1f=np.zeros((n, 3)), v1f=np.zeros((n, 3)), y1f=np.zeros((na, 3)), u1f=np.zeros((na, 3)),
    )
    out = _Out()
    for name, typ in _Out._fields_:
        setattr(out, name, r[name].ctypes.data_as(typ))
    fs = None if fsample is None else _c(fsample, np.int64)
    as_ = None if asample is None else _c(asample, np.int64)
    acc = None if agent_acc is None else _c(agent_acc, np.float64).reshape(na, 3)
    rin = None if rho_in is None else _c(rho_in, np.float64).reshape(n)
    rc = lib().orc_step_rho(ctypes.byref(_params(p, nbr_mode)), n, x.ctypes.data, v.ctypes.data, na, y.ctypes.data,
                            u.ctypes.data, None if fs is None else fs.ctypes.data, 0 if fs is None else fs.size,
                            None if as_ is None else as_.ctypes.data, 0 if as_ is None else as_.size,
                            None if acc is None else acc.ctypes.data, None if rin is None else rin.ctypes.data,
                            ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return r
