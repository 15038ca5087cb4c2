"""Thin ctypes binding of libnb (include/nb.h).

Argument marshalling only: every step of the pair-list build, force evaluation
and integration runs in libnb's HIP kernels.  torch supplies device memory (the
arenas and the caller's x/v/f tensors) and the HIP stream; there is no CPU
fallback -- importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnb.so")

NB_OK = 0
NB_ERR_ARG = -1
NB_ERR_BOX = -2
NB_ERR_CAPACITY = -3
NB_ERR_DEVICE = -4
NB_ERR_NONFINITE = -5
NB_ERR_BUFFER = -6
NB_ERR_STATE = -7

NB_COUL = {"none": 0, "rf": 1, "ewald": 2}
NB_LJ = {"single": 0, "lb": 1}
NB_POT_SHIFT = 1
NB_FP32_REDUCE = 2


class NbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnb error {code}: {msg}")
        self.code = code


class nb_params(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32),
        ("box", ctypes.c_double * 3),
        ("r_cut", ctypes.c_double),
        ("r_list", ctypes.c_double),
        ("coulomb", ctypes.c_int32),
        ("eps_r", ctypes.c_double),
        ("eps_rf", ctypes.c_double),
        ("ewald_beta", ctypes.c_double),
        ("lj", ctypes.c_int32),
        ("c6", ctypes.c_double),
        ("c12", ctypes.c_double),
        ("cluster", ctypes.c_int32),
        ("jtile", ctypes.c_int32),
        ("force_fixed_bits", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("r_inner", ctypes.c_double),
        ("nstprune", ctypes.c_int32),
        ("box_off", ctypes.c_double * 3),
        ("pme_grid", ctypes.c_int32 * 3),
        ("pme_order", ctypes.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libnb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnb.so not built at {path}; run python -m paper_1506_00716_amd.build")
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "nb_strerror": (ctypes.c_char_p, [i32]),
        "nb_last_error": (ctypes.c_char_p, [vp]),
        "nb_ctx_create": (i32, [ctypes.c_int, vp, P(vp)]),
        "nb_ctx_destroy": (i32, [vp]),
        "nb_arena_bytes": (i32, [P(nb_params), P(sz)]),
        "nb_sys_create": (i32, [vp, P(nb_params), vp, sz, P(vp)]),
        "nb_sys_destroy": (i32, [vp]),
        "nb_sys_needed_bytes": (i32, [vp, P(sz)]),
        "nb_sys_set_arena": (i32, [vp, vp, sz]),
        "nb_sys_set_particles": (i32, [vp, vp, vp, vp, vp]),
        "nb_build_pairlist": (i32, [vp, vp]),
        "nb_pairlist_export": (i32, [vp, vp, i64, P(i64)]),
        "nb_pairlist_stats": (i32, [vp, P(i64)]),
        "nb_compute_forces": (i32, [vp, vp, vp, vp, vp]),
        "nb_pme_forces": (i32, [vp, vp, vp, vp, vp]),
        "md_step": (i32, [vp, vp, vp, vp, f64, i32, i32, i32, vp, i32, P(i32)]),
        "nb_minimize": (i32, [vp, vp, vp, i32, f64, f64, i32, P(f64), P(i32)]),
        "nb_sys_get_step": (i32, [vp, P(i64)]),
        "nb_sys_set_step": (i32, [vp, i64]),
        "nb_state_bytes": (i32, [vp, P(sz)]),
        "nb_state_export": (i32, [vp, vp, vp, vp, sz]),
        "nb_state_import": (i32, [vp, vp, vp, vp, sz]),
        "nb_sys_ewald_fit_error": (i32, [vp, P(f64)]),
        "nb_sys_set_timing": (i32, [vp, i32]),
        "nb_sys_get_timings": (i32, [vp, P(f64)]),
        "nb_sys_set_build_checks": (i32, [vp, i32]),
        "nb_sys_buffer_stats": (i32, [vp, P(f64)]),
        "nb_ens_arena_bytes": (i32, [i32, P(sz)]),
        "nb_ens_create": (i32, [vp, i32, vp, sz, P(vp)]),
        "nb_ens_destroy": (i32, [vp]),
        "nb_ens_add": (i32, [vp, vp, vp, vp, vp]),
        "nb_ens_remove": (i32, [vp, vp]),
        "nb_ens_size": (i32, [vp, P(i32)]),
        "nb_ens_member_index": (i32, [vp, vp, P(i32)]),
        "nb_ens_step": (i32, [vp, i32, f64, i32, i32, vp]),
        "nb_autotune": (i32, [vp, vp, vp, vp, sz, P(i32), i32, P(i32), i32, i32, P(i32), P(i32), P(f64)]),
        "nb_srv_create": (i32, [vp, vp, sz, vp, sz, i32, f64, i32, i32, P(vp)]),
        "nb_srv_submit": (i32, [vp, P(nb_params), vp, vp, vp, vp, vp, vp, i32, P(ctypes.c_uint64)]),
        "nb_srv_poll": (i32, [vp, ctypes.c_uint64, P(i32), P(f64), P(f64), P(i32)]),
        "nb_srv_fetch": (i32, [vp, ctypes.c_uint64, vp, vp]),
        "nb_srv_release": (i32, [vp, ctypes.c_uint64]),
        "nb_srv_wait_idle": (i32, [vp, f64]),
        "nb_srv_stats": (i32, [vp, P(f64)]),
        "nb_srv_destroy": (i32, [vp]),
        "nb_compute_forces_noalloc": (i32, [vp, P(nb_params), vp, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(code: int, ctx=None):
    if code != NB_OK:
        L = load()
        msg = L.nb_last_error(ctx).decode() if ctx is not None else L.nb_last_error(None).decode()
        raise NbError(code, msg or L.nb_strerror(code).decode())


def make_params(n_atoms: int, box, model, cluster: int = 0, jtile: int = 0,
                fp32_reduce: bool = False, force_fixed_bits: int = 0, r_inner: float = 0.0,
                nstprune: int = 0, box_off=None) -> nb_params:
    p = nb_params()
    p.n_atoms = int(n_atoms)
    for k in range(3):
        p.box[k] = float(box[k])
    p.r_cut = float(model.r_cut)
    p.r_list = float(model.r_list)
    p.coulomb = NB_COUL[model.coulomb]
    p.eps_r = float(model.eps_r)
    p.eps_rf = float(model.eps_rf)
    p.ewald_beta = float(model.ewald_beta)
    p.lj = NB_LJ[model.lj]
    p.c6 = float(model.c6)
    p.c12 = float(model.c12)
    p.cluster = int(cluster)
    p.jtile = int(jtile)
    p.force_fixed_bits = int(force_fixed_bits)
    p.flags = (NB_POT_SHIFT if model.pot_shift else 0) | (NB_FP32_REDUCE if fp32_reduce else 0)
    p.r_inner = float(r_inner)
    p.nstprune = int(nstprune)
    if box_off is not None:
        for k in range(3):
            p.box_off[k] = float(box_off[k])
    grid = getattr(model, "pme_grid", None)
    if grid is not None:
        for k in range(3):
            p.pme_grid[k] = int(grid[k])
        p.pme_order = int(getattr(model, "pme_order", 4))
    return p


def pme_grid_for(box, box_off=None, spacing: float = 0.12):
    """PME grid points along each lattice vector for at most `spacing` nm
    between points (the lengths of a, b, c of a lower-triangular box)."""
    off = [0.0, 0.0, 0.0] if box_off is None else [float(v) for v in box_off]
    lengths = (float(box[0]), math.hypot(off[0], float(box[1])), math.sqrt(off[1] ** 2 + off[2] ** 2 + float(box[2]) ** 2))
    return tuple(max(4, int(math.ceil(v / spacing - 1e-9))) for v in lengths)


def arena_bytes(params: nb_params) -> int:
    L = load()
    b = ctypes.c_size_t()
    _check(L.nb_arena_bytes(ctypes.byref(params), ctypes.byref(b)))
    return int(b.value)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(t.data_ptr()))


def _hostp(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


class Context:
    """A libnb context on `device` bound to torch's current HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        L = load()
        h = ctypes.c_void_p()
        _check(L.nb_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().nb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """One periodic system: a device arena plus libnb handles."""

    def __init__(self, ctx: Context, sysm, cluster: int = 0, jtile: int = 0,
                 fp32_reduce: bool = False, force_fixed_bits: int = 0, model=None,
                 r_inner: float = 0.0, nstprune: int = 0):
        torch = ctx.torch
        self.ctx = ctx
        self.model = model or sysm.model
        self.n = sysm.n
        self.params = make_params(sysm.n, sysm.box, self.model, cluster, jtile, fp32_reduce,
                                  force_fixed_bits, r_inner, nstprune, getattr(sysm, "box_off", None))
        L = load()
        nbytes = arena_bytes(self.params)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=ctx.device)
        h = ctypes.c_void_p()
        _check(L.nb_sys_create(ctx.h, ctypes.byref(self.params), _ptr(self.arena), nbytes,
                               ctypes.byref(h)), ctx.h)
        self.h = h
        q = np.ascontiguousarray(sysm.q, dtype=np.float64)
        sg = np.ascontiguousarray(sysm.sigma, dtype=np.float64)
        ep = np.ascontiguousarray(sysm.epsilon, dtype=np.float64)
        ms = np.ascontiguousarray(sysm.mass, dtype=np.float64)
        _check(L.nb_sys_set_particles(h, _hostp(q), _hostp(sg), _hostp(ep), _hostp(ms)), ctx.h)

    # -- helpers ----------------------------------------------------------
    def _call_growing(self, fn):
        """Run fn(); on NB_ERR_CAPACITY move to a larger arena and retry."""
        for _ in range(4):
            code = fn()
            if code != NB_ERR_CAPACITY:
                _check(code, self.ctx.h)
                return
            self._grow()
        raise NbError(NB_ERR_CAPACITY, "arena growth did not converge")

    def _grow(self):
        """Move the system to an arena of the size the library asked for."""
        L = load()
        need = ctypes.c_size_t()
        _check(L.nb_sys_needed_bytes(self.h, ctypes.byref(need)), self.ctx.h)
        self.arena = self.ctx.torch.empty(int(need.value), dtype=self.ctx.torch.uint8, device=self.ctx.device)
        _check(L.nb_sys_set_arena(self.h, _ptr(self.arena), int(need.value)), self.ctx.h)

    def build_pairlist(self, x):
        L = load()
        self._call_growing(lambda: L.nb_build_pairlist(self.h, _ptr(x)))

    def export_pairs(self) -> np.ndarray:
        L = load()
        n = ctypes.c_int64()
        _check(L.nb_pairlist_export(self.h, None, 0, ctypes.byref(n)), self.ctx.h)
        out = np.zeros((max(n.value, 1), 2), dtype=np.int32)
        _check(L.nb_pairlist_export(self.h, _hostp(out), n.value, ctypes.byref(n)), self.ctx.h)
        return out[: n.value]

    def stats(self) -> dict:
        L = load()
        a = (ctypes.c_int64 * 10)()
        _check(L.nb_pairlist_stats(self.h, a), self.ctx.h)
        keys = ["clusters", "entries", "cluster_pairs", "atom_pairs_rlist", "evaluated_pairs",
                "items", "groups", "slots", "pairs_rcut", "candidates"]
        return dict(zip(keys, [int(v) for v in a]))

    def compute_forces(self, x, f, energies: bool = True):
        L = load()
        e = np.zeros(2)
        w = np.zeros(9)
        if energies:
            self._call_growing(lambda: L.nb_compute_forces(self.h, _ptr(x), _ptr(f), _hostp(e), _hostp(w)))
            return e, w.reshape(3, 3)
        self._call_growing(lambda: L.nb_compute_forces(self.h, _ptr(x), _ptr(f), None, None))
        return None, None

    def pme_forces(self, x, f, energies: bool = True):
        """Reciprocal-space Ewald forces alone (a system with PME): f receives
        them; returns (E_recip + E_self + E_background, virial [3,3]) or
        (None, None)."""
        L = load()
        if energies:
            e = np.zeros(1)
            w = np.zeros(9)
            _check(L.nb_pme_forces(self.h, _ptr(x), _ptr(f), _hostp(e), _hostp(w)), self.ctx.h)
            return float(e[0]), w.reshape(3, 3)
        _check(L.nb_pme_forces(self.h, _ptr(x), _ptr(f), None, None), self.ctx.h)
        return None, None

    def md_step(self, x, v, f, dt: float, n_steps: int, nstlist: int = 10, nstenergy: int = 0):
        """n_steps velocity-Verlet steps; if a rebuild runs out of list capacity the
        library stops at the last full step, and the remaining steps run again on
        a grown arena."""
        L = load()
        rows_cap = (n_steps // nstenergy + 1) if nstenergy > 0 else 0
        out = []
        left = int(n_steps)
        for _ in range(5):
            tr = np.zeros((max(rows_cap, 1), 5))
            nr = ctypes.c_int32()
            step0 = self.step
            code = L.md_step(self.h, _ptr(x), _ptr(v), _ptr(f), float(dt), left, int(nstlist), int(nstenergy),
                             _hostp(tr) if rows_cap else None, rows_cap, ctypes.byref(nr))
            out.append(tr[: nr.value].copy())
            done = self.step - step0
            left -= done
            if code != NB_ERR_CAPACITY:
                _check(code, self.ctx.h)
                return np.concatenate(out) if out else tr[:0]
            if left == 0:
                # every step ran: the overflow was found after the fact (build
                # checks off), so the trajectory is not valid and cannot resume
                _check(code, self.ctx.h)
            self._grow()
        raise NbError(NB_ERR_CAPACITY, "arena growth did not converge")

    def minimize(self, x, f, n_iter: int = 500, f_tol: float = 1000.0, max_disp: float = 0.002,
                 nstlist: int = 10):
        L = load()
        fm = ctypes.c_double()
        it = ctypes.c_int32()
        self._call_growing(lambda: L.nb_minimize(self.h, _ptr(x), _ptr(f), int(n_iter), float(f_tol),
                                                 float(max_disp), int(nstlist), ctypes.byref(fm),
                                                 ctypes.byref(it)))
        return fm.value, it.value

    @property
    def step(self) -> int:
        s = ctypes.c_int64()
        _check(load().nb_sys_get_step(self.h, ctypes.byref(s)))
        return int(s.value)

    @step.setter
    def step(self, v: int):
        _check(load().nb_sys_set_step(self.h, int(v)))

    def state_export(self, x, v) -> bytes:
        L = load()
        n = ctypes.c_size_t()
        _check(L.nb_state_bytes(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(L.nb_state_export(self.h, _ptr(x), _ptr(v), buf, n.value), self.ctx.h)
        return buf.raw

    def state_import(self, x, v, blob: bytes):
        L = load()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(L.nb_state_import(self.h, _ptr(x), _ptr(v), buf, len(blob)), self.ctx.h)

    def set_timing(self, on: bool = True, every: int = 1):
        """HIP-event timers of md_step; every = k times one of every k force
        launches and rebuilds."""
        _check(load().nb_sys_set_timing(self.h, int(every) if on else 0))

    def timings(self) -> dict:
        a = (ctypes.c_double * 6)()
        _check(load().nb_sys_get_timings(self.h, a))
        return {"force_ms": a[0], "force_launches": int(a[1]), "build_ms": a[2], "builds": int(a[3]),
                "md_ms": a[4], "md_calls": int(a[5])}

    def buffer_stats(self) -> dict:
        a = (ctypes.c_double * 4)()
        _check(load().nb_sys_buffer_stats(self.h, a), self.ctx.h)
        return {"max_displacement": a[0], "unsafe_lifetimes": int(a[1]),
                "prune_max_displacement": a[2], "unsafe_prune_intervals": int(a[3])}

    def set_build_checks(self, on: bool):
        _check(load().nb_sys_set_build_checks(self.h, 1 if on else 0))

    def autotune(self, x, f, clusters=(4, 8), jtiles=(8, 16, 32, 64), reps: int = 5):
        """Fastest (cluster, jtile) for this system's model at positions x."""
        L = load()
        torch = self.ctx.torch
        need = 0
        for m in clusters:
            for j in jtiles:
                need = max(need, arena_bytes(make_params(self.n, self.params.box, self.model, m, j,
                                                         box_off=self.params.box_off)))
        scratch = torch.empty(int(need * 1.5), dtype=torch.uint8, device=self.ctx.device)
        cl = (ctypes.c_int32 * len(clusters))(*clusters)
        jt = (ctypes.c_int32 * len(jtiles))(*jtiles)
        bc, bj, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(L.nb_autotune(self.h, _ptr(x), _ptr(f), _ptr(scratch), scratch.numel(), cl, len(clusters),
                             jt, len(jtiles), reps, ctypes.byref(bc), ctypes.byref(bj), ctypes.byref(us)),
               self.ctx.h)
        return bc.value, bj.value, us.value

    def ewald_fit_error(self) -> float:
        e = ctypes.c_double()
        _check(load().nb_sys_ewald_fit_error(self.h, ctypes.byref(e)))
        return e.value

    def close(self):
        if getattr(self, "h", None):
            load().nb_sys_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """A batch of Systems advanced together (one launch per kernel per step)."""

    def __init__(self, ctx: Context, max_systems: int):
        L = load()
        self.ctx = ctx
        b = ctypes.c_size_t()
        _check(L.nb_ens_arena_bytes(int(max_systems), ctypes.byref(b)))
        self.arena = ctx.torch.empty(int(b.value), dtype=ctx.torch.uint8, device=ctx.device)
        h = ctypes.c_void_p()
        _check(L.nb_ens_create(ctx.h, int(max_systems), _ptr(self.arena), int(b.value), ctypes.byref(h)), ctx.h)
        self.h = h
        self.members = []

    def add(self, system: System, x, v, f):
        _check(load().nb_ens_add(self.h, system.h, _ptr(x), _ptr(v), _ptr(f)), self.ctx.h)
        self.members.append((system, x, v, f))

    def remove(self, system: System):
        _check(load().nb_ens_remove(self.h, system.h), self.ctx.h)
        self.members = [m for m in self.members if m[0] is not system]

    def size(self) -> int:
        n = ctypes.c_int32()
        _check(load().nb_ens_size(self.h, ctypes.byref(n)))
        return n.value

    def index_of(self, system: System) -> int:
        i = ctypes.c_int32()
        _check(load().nb_ens_member_index(self.h, system.h, ctypes.byref(i)), self.ctx.h)
        return i.value

    def step(self, n_steps: int, dt: float, nstlist: int = 10, use_graph: bool = True,
             energies: bool = False):
        L = load()
        n = len(self.members)
        out = np.zeros((max(n, 1), 3)) if energies else None
        _check(L.nb_ens_step(self.h, int(n_steps), float(dt), int(nstlist), 1 if use_graph else 0,
                             _hostp(out) if energies else None), self.ctx.h)
        if energies:
            # rows are in the ensemble's internal order: map back to insertion order
            res = np.zeros((n, 3))
            for k, (system, _, _, _) in enumerate(self.members):
                res[k] = out[self.index_of(system)]
            return res
        return None

    def close(self):
        if getattr(self, "h", None):
            load().nb_ens_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_MAX_BYTES = 64 << 20


def compute_forces_noalloc(ctx: Context, sysm, x, f, energies: bool = True, cluster: int = 0,
                           jtile: int = 0, fp32_reduce: bool = False, force_fixed_bits: int = 0,
                           model=None):
    """List build + forces for one system in the library's fixed device array
    (nb_compute_forces_noalloc): no arena, no system handle.  Returns
    (energies, virial) or (None, None)."""
    L = load()
    p = make_params(sysm.n, sysm.box, model or sysm.model, cluster, jtile, fp32_reduce, force_fixed_bits,
                    box_off=getattr(sysm, "box_off", None))
    q = np.ascontiguousarray(sysm.q, dtype=np.float64)
    sg = np.ascontiguousarray(sysm.sigma, dtype=np.float64)
    ep = np.ascontiguousarray(sysm.epsilon, dtype=np.float64)
    e = np.zeros(2)
    w = np.zeros(9)
    _check(L.nb_compute_forces_noalloc(ctx.h, ctypes.byref(p), _hostp(q), _hostp(sg), _hostp(ep), _ptr(x),
                                       _ptr(f), _hostp(e) if energies else None,
                                       _hostp(w) if energies else None), ctx.h)
    return (e, w.reshape(3, 3)) if energies else (None, None)


def device_state(sysm, device="cuda:0"):
    """x (FP64), v (FP64), f (FP32) device tensors of a generated system."""
    import torch
    x = torch.tensor(np.ascontiguousarray(sysm.x), dtype=torch.float64, device=device)
    v = torch.tensor(np.ascontiguousarray(sysm.v if sysm.v is not None else np.zeros_like(sysm.x)),
                     dtype=torch.float64, device=device)
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device=device)
    return x, v, f


class Server:
    """Continuous-batching MD job server on one GPU (native host thread in libnb)."""

    STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "rejected"}

    def __init__(self, ctx: Context, pool_bytes: int, max_slots: int = 64, dt: float = 0.002,
                 nstlist: int = 10, use_graph: bool = True):
        L = load()
        torch = ctx.torch
        self.ctx = ctx
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=ctx.device)
        b = ctypes.c_size_t()
        _check(L.nb_ens_arena_bytes(int(max_slots), ctypes.byref(b)))
        self.ens_arena = torch.empty(int(b.value), dtype=torch.uint8, device=ctx.device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(L.nb_srv_create(ctx.h, _ptr(self.pool), int(pool_bytes), _ptr(self.ens_arena), int(b.value),
                               int(max_slots), float(dt), int(nstlist), 1 if use_graph else 0,
                               ctypes.byref(h)), ctx.h)
        self.h = h
        self._keep = {}

    def submit(self, sysm, n_steps: int, cluster: int = 0, jtile: int = 0) -> int:
        L = load()
        p = make_params(sysm.n, sysm.box, sysm.model, cluster, jtile, box_off=getattr(sysm, "box_off", None))
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in
                (sysm.x, sysm.v if sysm.v is not None else np.zeros_like(sysm.x), sysm.q, sysm.sigma,
                 sysm.epsilon, sysm.mass)]
        jid = ctypes.c_uint64()
        _check(L.nb_srv_submit(self.h, ctypes.byref(p), *[_hostp(a) for a in arrs], int(n_steps),
                               ctypes.byref(jid)))
        return int(jid.value)

    def poll(self, job_id: int) -> dict:
        st = ctypes.c_int32()
        t = (ctypes.c_double * 3)()
        e = (ctypes.c_double * 3)()
        err = ctypes.c_int32()
        _check(load().nb_srv_poll(self.h, ctypes.c_uint64(job_id), ctypes.byref(st), t, e, ctypes.byref(err)))
        return {"state": self.STATES[st.value], "t_submit": t[0], "t_admit": t[1], "t_done": t[2],
                "energies": list(e), "error": err.value}

    def fetch(self, job_id: int, n_atoms: int):
        x = np.zeros((n_atoms, 3))
        v = np.zeros((n_atoms, 3))
        _check(load().nb_srv_fetch(self.h, ctypes.c_uint64(job_id), _hostp(x), _hostp(v)))
        return x, v

    def release(self, job_id: int):
        _check(load().nb_srv_release(self.h, ctypes.c_uint64(job_id)))

    def wait_idle(self, timeout: float = 600.0):
        _check(load().nb_srv_wait_idle(self.h, float(timeout)))

    def stats(self) -> dict:
        a = (ctypes.c_double * 8)()
        _check(load().nb_srv_stats(self.h, a))
        keys = ["atom_steps", "done", "failed", "rejected", "busy_s", "uptime_s", "running", "queued"]
        return dict(zip(keys, list(a)))

    def close(self):
        if getattr(self, "h", None):
            load().nb_srv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
