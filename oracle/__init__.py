"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports, links or
calls anything here, and nothing here imports the product package.

All functions take numpy arrays in the layout of ``paper_1506_00716_amd.inputs``
(positions [N,3] FP64, nm) and return FP64 numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Compile flags: FP64, no contraction of a*b+c into FMA (the pair-set criterion
# must be evaluated with separately rounded operations), OpenMP over atoms.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

_COUL = {"none": 0, "rf": 1, "ewald": 2}
_LJ = {"single": 0, "lb": 1}

_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def configure(L):
    """Declare the C signatures on a loaded oracle library (ctypes.CDLL)."""
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.oracle_pairs.restype = i64
    L.oracle_pairs.argtypes = [i32, dp, dp, dp, f64, ip, i64, i32]
    model = [f64, i32, f64, f64, f64, i32, f64, f64, i32, i32]
    L.oracle_forces.restype = ctypes.c_int
    L.oracle_forces.argtypes = [i32, dp, dp, dp, dp, dp, dp] + model + [dp, dp, dp]
    L.oracle_forces_subset.restype = ctypes.c_int
    L.oracle_forces_subset.argtypes = [i32, dp, dp, dp, dp, dp, dp] + model + [ip, i32, dp, dp]
    L.oracle_md.restype = ctypes.c_int
    L.oracle_md.argtypes = [i32, dp, dp, dp, dp, dp, dp, dp, dp] + model + [f64, i32, dp]
    L.oracle_num_threads.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = configure(ctypes.CDLL(_LIB))
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _box(box, box_off=None):
    """(box[6], invbox[3]): the diagonal a_x, b_y, c_z, then the off-diagonal
    b_x, c_x, c_y of a lower-triangular box (zeros: rectangular)."""
    box = _f64(box).reshape(3)
    off = np.zeros(3) if box_off is None else _f64(box_off).reshape(3)
    # 1/L computed once in FP64 and used by every pair (and by the GPU side).
    return np.concatenate([box, off]), _f64(1.0 / box)


def _sys_box(sysm):
    return _box(sysm.box, getattr(sysm, "box_off", None))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def pairs(x, box, r_list, nthreads: int = 0, box_off=None) -> np.ndarray:
    """Canonical pair set: int32 [P, 2], i < j, sorted lexicographically."""
    x = _f64(x, (-1, 3))
    box, inv = _box(box, box_off)
    n = x.shape[0]
    total = lib().oracle_pairs(n, _dp(x), _dp(box), _dp(inv), float(r_list), None, 0, nthreads)
    if total < 0:
        raise ValueError("oracle_pairs: bad arguments")
    out = np.zeros((max(total, 1), 2), dtype=np.int32)
    got = lib().oracle_pairs(n, _dp(x), _dp(box), _dp(inv), float(r_list), _ip(out), total, nthreads)
    assert got == total
    return out[:total]


def _model_args(model, c6=None, c12=None):
    return [float(model.r_cut), _COUL[model.coulomb], float(model.eps_r), float(model.eps_rf),
            float(model.ewald_beta), _LJ[model.lj],
            float(model.c6 if c6 is None else c6), float(model.c12 if c12 is None else c12),
            1 if model.pot_shift else 0]


def forces(sysm, x=None, model=None, nthreads: int = 0):
    """Returns (f [N,3], energies (E_LJ, E_coul), virial [3,3])."""
    model = model or sysm.model
    x = _f64(sysm.x if x is None else x, (-1, 3))
    n = x.shape[0]
    box, inv = _sys_box(sysm)
    q = _f64(sysm.q)
    sig, eps = _f64(sysm.sigma), _f64(sysm.epsilon)
    f = np.zeros((n, 3))
    e = np.zeros(2)
    w = np.zeros(9)
    rc = lib().oracle_forces(n, _dp(x), _dp(q), _dp(sig), _dp(eps), _dp(box), _dp(inv),
                             *_model_args(model), nthreads, _dp(f), _dp(e), _dp(w))
    if rc != 0:
        raise ValueError("oracle_forces failed")
    return f, e, w.reshape(3, 3)


def forces_subset(sysm, idx, x=None, model=None, nthreads: int = 0):
    """Forces (and half pair energies) on the atoms idx only."""
    model = model or sysm.model
    x = _f64(sysm.x if x is None else x, (-1, 3))
    n = x.shape[0]
    box, inv = _sys_box(sysm)
    q = _f64(sysm.q)
    sig, eps = _f64(sysm.sigma), _f64(sysm.epsilon)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    f = np.zeros((idx.shape[0], 3))
    e = np.zeros((idx.shape[0], 2))
    rc = lib().oracle_forces_subset(n, _dp(x), _dp(q), _dp(sig), _dp(eps), _dp(box), _dp(inv),
                                    *_model_args(model), nthreads, _ip(idx), idx.shape[0],
                                    _dp(f), _dp(e))
    if rc != 0:
        raise ValueError("oracle_forces_subset failed")
    return f, e


def md(sysm, x, v, dt: float, nsteps: int, model=None, nthreads: int = 0):
    """FP64 velocity Verlet with all-pairs forces.  Returns (x, v, trace[nsteps,4])."""
    model = model or sysm.model
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    n = x.shape[0]
    box, inv = _sys_box(sysm)
    q = _f64(sysm.q)
    m = _f64(sysm.mass)
    sig, eps = _f64(sysm.sigma), _f64(sysm.epsilon)
    tr = np.zeros((max(nsteps, 1), 4))
    rc = lib().oracle_md(n, _dp(x), _dp(v), _dp(m), _dp(q), _dp(sig), _dp(eps), _dp(box), _dp(inv),
                         *_model_args(model), nthreads, float(dt), int(nsteps), _dp(tr))
    if rc != 0:
        raise ValueError("oracle_md failed")
    return x, v, tr[:nsteps]
