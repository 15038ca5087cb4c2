"""The C ABI library: it loads, exports every function include/nb.h declares,
and its host-only calls validate parameters (no device needed)."""
import ctypes
import os
import re

import pytest

from paper_1506_00716_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             src, flags=re.M):
            names.add(m.group(1))
    names.discard("if")
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("nb_build_pairlist", "nb_compute_forces", "md_step", "nb_pairlist_export"):
        assert must in names


def test_library_exports_every_declared_symbol(nbmod):
    lib = ctypes.CDLL(nbmod.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_codes(nbmod):
    L = nbmod.load()
    for code in range(-7, 1):
        s = L.nb_strerror(code)
        assert s and len(s) >= 2
    assert L.nb_strerror(-99) == b"unknown status"


def test_arena_bytes_validates(nbmod):
    s = inputs.small_rf()
    p = nbmod.make_params(s.n, s.box, s.model)
    assert nbmod.arena_bytes(p) > 1_000_000
    L = nbmod.load()
    b = ctypes.c_size_t()
    bad = nbmod.make_params(s.n, [1.9, 3.0, 3.0], s.model)  # r_list 1.0 >= L/2 = 0.95
    assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_BOX
    bad = nbmod.make_params(s.n, s.box, s.model, cluster=3)
    assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_ARG
    bad = nbmod.make_params(0, s.box, s.model)
    assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_ARG
    m = inputs.Model(r_cut=1.0, r_list=0.9, coulomb="rf")
    bad = nbmod.make_params(s.n, s.box, m)
    assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_ARG
    m = inputs.Model(r_cut=0.9, r_list=1.0, coulomb="ewald", ewald_beta=0.0)
    bad = nbmod.make_params(s.n, s.box, m)
    assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_ARG
    assert L.nb_arena_bytes(None, ctypes.byref(b)) == nbmod.NB_ERR_ARG
    # triclinic boxes: the dodecahedron is accepted, skews beyond half an edge are not
    d = 3.0
    ok = nbmod.make_params(s.n, [d, d, d / 2 ** 0.5], s.model, box_off=[0.0, d / 2, d / 2])
    assert L.nb_arena_bytes(ctypes.byref(ok), ctypes.byref(b)) == nbmod.NB_OK
    for off in ([1.6, 0.0, 0.0], [0.0, -1.6, 0.0], [0.0, 0.0, 1.6], [float("nan"), 0.0, 0.0]):
        bad = nbmod.make_params(s.n, [3.0, 3.0, 3.0], s.model, box_off=off)
        assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_BOX
    # dynamic pruning: r_inner within [r_cut, r_list] and an interval >= 1
    ok = nbmod.make_params(s.n, s.box, s.model, r_inner=0.95, nstprune=4)
    assert L.nb_arena_bytes(ctypes.byref(ok), ctypes.byref(b)) == nbmod.NB_OK
    for r_inner, nstprune in ((0.85, 4), (1.05, 4), (0.95, 0), (-0.5, 1)):
        bad = nbmod.make_params(s.n, s.box, s.model, r_inner=r_inner, nstprune=nstprune)
        assert L.nb_arena_bytes(ctypes.byref(bad), ctypes.byref(b)) == nbmod.NB_ERR_ARG


def test_pme_parameters_validated(nbmod):
    L = nbmod.load()
    b = ctypes.c_size_t()

    def code(model):
        p = nbmod.make_params(3000, [3.0, 3.1, 3.2], model)
        return L.nb_arena_bytes(ctypes.byref(p), ctypes.byref(b))

    ew = dict(r_cut=0.9, r_list=1.0, coulomb="ewald", ewald_beta=3.12)
    assert code(inputs.Model(**ew, pme_grid=(24, 26, 27), pme_order=4)) == nbmod.NB_OK
    small = b.value
    assert code(inputs.Model(**ew)) == nbmod.NB_OK
    assert small > b.value  # the grids live in the arena
    assert code(inputs.Model(**ew, pme_grid=(6, 6, 6), pme_order=6)) == nbmod.NB_OK
    assert code(inputs.Model(**ew, pme_grid=(256, 4, 4), pme_order=4)) == nbmod.NB_OK
    for grid, order in (((24, 26, 3), 4), ((5, 24, 24), 6), ((257, 24, 24), 4), ((24, 24, 24), 5),
                        ((24, 0, 24), 4), ((24, 24, -8), 4)):
        assert code(inputs.Model(**ew, pme_grid=grid, pme_order=order)) == nbmod.NB_ERR_ARG, (grid, order)
    rf = inputs.Model(r_cut=0.9, r_list=1.0, coulomb="rf", pme_grid=(24, 24, 24))
    assert code(rf) == nbmod.NB_ERR_ARG


def test_pme_grid_for_spacing(nbmod):
    assert nbmod.pme_grid_for([6.2, 6.2, 6.2]) == (52, 52, 52)
    box, off = inputs.dodecahedron_box(6.2)
    # every lattice vector of the dodecahedron has length d
    assert nbmod.pme_grid_for(box, off) == (52, 52, 52)


def test_arena_grows_with_system_size(nbmod):
    small = nbmod.make_params(2700, [3.0] * 3, inputs.MODEL_RF)
    big = nbmod.make_params(24000, [6.2] * 3, inputs.MODEL_EWALD)
    assert nbmod.arena_bytes(big) > 4 * nbmod.arena_bytes(small)
    # every cluster size has a layout
    for m in (1, 4, 8):
        assert nbmod.arena_bytes(nbmod.make_params(2700, [3.0] * 3, inputs.MODEL_RF, cluster=m)) > 0


def test_null_handles_rejected(nbmod):
    L = nbmod.load()
    assert L.nb_sys_destroy(None) == nbmod.NB_ERR_ARG
    assert L.nb_ctx_destroy(None) == nbmod.NB_ERR_ARG
    assert L.nb_build_pairlist(None, None) == nbmod.NB_ERR_ARG
    assert L.nb_compute_forces(None, None, None, None, None) == nbmod.NB_ERR_ARG
    assert L.md_step(None, None, None, None, 0.002, 1, 10, 0, None, 0, None) == nbmod.NB_ERR_ARG
