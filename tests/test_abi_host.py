"""The C-ABI library loads, exports every function include/ocn.h declares, and
validates arguments on the host (no GPU call is made here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2309_06662_amd import inputs, ocn

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ocn.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ocn_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(ocn.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    L = ocn.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.ocn_abi_version() == 3


def _grid(w, **over):
    inp = inputs.make_inputs(w)
    desc, keep = ocn.grid_desc(w, inp["dz"], inp["kbottom"])
    for k, v in over.items():
        setattr(desc, k, v)
    h = C.c_void_p()
    rc = ocn.lib().ocn_grid_create(C.byref(desc), C.byref(h))
    return rc, h, keep


def test_grid_create_validates_arguments():
    w = inputs.BETA_BASIN_64.replace(nx=8, ny=6, nz=4)
    rc, h, _ = _grid(w)
    assert rc == ocn.OCN_OK
    ocn.lib().ocn_grid_destroy(h)
    for bad in ({"nx": 0}, {"halo": 2}, {"halo": 9}, {"coords": 5}, {"reserved": 1}, {"dx": -1.0}):
        rc, h, _ = _grid(w, **bad)
        assert rc == ocn.OCN_E_INVALID, bad
        assert ocn.lib().ocn_last_error()
    ll = inputs.LATLON_QUARTER.replace(nx=16, ny=10, nz=4, dx=22.5, dy=16.0, bathymetry="flat")
    rc, h, _ = _grid(ll, periodic_y=1)
    assert rc == ocn.OCN_E_INVALID
    rc, h, _ = _grid(ll.replace(y0=-89.0))
    assert rc == ocn.OCN_E_INVALID
    assert ocn.lib().ocn_grid_create(None, C.byref(C.c_void_p())) == ocn.OCN_E_INVALID


def test_arena_size_scales_with_precision_and_validates_params():
    w = inputs.BETA_BASIN_64.replace(nx=400, ny=300, nz=10)   # sizes only: nothing is allocated
    rc, h, keep = _grid(w)
    assert rc == 0
    n64, n32 = C.c_size_t(), C.c_size_t()
    L = ocn.lib()
    p = ocn.params(w, "fp64")
    assert L.ocn_state_arena_bytes(h, C.byref(p), C.byref(n64)) == 0
    p32 = ocn.params(w, "fp32")
    assert L.ocn_state_arena_bytes(h, C.byref(p32), C.byref(n32)) == 0
    # nine 3D fields change element size; the FP64 2D fields and tables do not
    cells = 400 * 300 * 10
    assert n64.value >= 9 * cells * 8 + 22 * 400 * 300 * 8
    assert n64.value - n32.value >= 9 * cells * 4
    assert n32.value < n64.value
    # salinity adds four 3D fields (S, S*, and the two AB2 histories of S)
    ns = C.c_size_t()
    ps = ocn.params(w.replace(salinity=True), "fp64")
    assert ps.salinity == 1 and list(ps.eos) == list(w.eos)
    assert L.ocn_state_arena_bytes(h, C.byref(ps), C.byref(ns)) == 0
    assert ns.value - n64.value >= 4 * cells * 8
    bad = ocn.params(w.replace(salinity=True), "fp64")
    bad.eos[3] = float("nan")
    assert L.ocn_state_arena_bytes(h, C.byref(bad), C.byref(ns)) == ocn.OCN_E_INVALID
    bad.salinity = 2
    bad.eos[3] = 0.0
    assert L.ocn_state_arena_bytes(h, C.byref(bad), C.byref(ns)) == ocn.OCN_E_INVALID
    bad = ocn.params(w, "fp64")
    bad.n_substeps = 0
    assert L.ocn_state_arena_bytes(h, C.byref(bad), C.byref(n64)) == ocn.OCN_E_INVALID
    bad = ocn.params(w, "fp64")
    bad.dt = -5.0
    assert L.ocn_state_arena_bytes(h, C.byref(bad), C.byref(n64)) == ocn.OCN_E_INVALID
    for name, value in (("chi", float("nan")), ("g", 0.0), ("g", float("inf")), ("alpha", float("nan")),
                        ("t_ref", float("inf")), ("restore_tau", float("nan")), ("momentum_form", 2),
                        ("pgf_weight", 1.5), ("reserved2", 1)):
        bad = ocn.params(w, "fp64")
        setattr(bad, name, value)
        assert L.ocn_state_arena_bytes(h, C.byref(bad), C.byref(n64)) == ocn.OCN_E_INVALID, name
    vi = ocn.params(w.replace(momentum_form="vector_invariant"), "fp64")
    assert vi.momentum_form == 1 and L.ocn_state_arena_bytes(h, C.byref(vi), C.byref(n64)) == 0
    # 128 levels is the most a state may have
    for nz, rc_expect in ((128, 0), (129, ocn.OCN_E_UNSUPPORTED)):
        wz = w.replace(nx=8, ny=6, nz=nz)
        rc, hz, keepz = _grid(wz)
        assert rc == 0
        pz = ocn.params(wz, "fp64")
        assert L.ocn_state_arena_bytes(hz, C.byref(pz), C.byref(n64)) == rc_expect, nz
        L.ocn_grid_destroy(hz)
    # state calls reject NULL handles without touching a device
    assert L.ocn_step(None, 1) == ocn.OCN_E_INVALID
    assert L.ocn_synchronize(None) == ocn.OCN_E_INVALID
    assert L.ocn_state_init(h, C.byref(p), None, 0, None, C.byref(C.c_void_p())) == ocn.OCN_E_INVALID
    L.ocn_grid_destroy(h)


def test_ensemble_arena_and_argument_checks():
    L = ocn.lib()
    ws = [inputs.BETA_BASIN_64.replace(nx=20 + 7 * m, ny=15 + 3 * m, nz=4 + m) for m in range(3)]
    grids = [ocn.Grid(w, inputs.layer_thickness(w), inputs.wet_layers(w)) for w in ws]
    arr = (C.c_void_p * 3)(*[g.handle.value for g in grids])
    p = ocn.params(ws[0], "fp32")
    total, one = C.c_size_t(), C.c_size_t()
    assert L.ocn_ensemble_arena_bytes(arr, 3, C.byref(p), C.byref(total)) == 0
    parts = 0
    for g in grids:
        assert L.ocn_state_arena_bytes(g.handle, C.byref(p), C.byref(one)) == 0
        parts += one.value
    assert total.value > parts  # members plus the member table and tile tables
    assert L.ocn_ensemble_arena_bytes(arr, 0, C.byref(p), C.byref(total)) == ocn.OCN_E_INVALID
    bad = (C.c_void_p * 2)(grids[0].handle.value, None)
    assert L.ocn_ensemble_arena_bytes(bad, 2, C.byref(p), C.byref(total)) == ocn.OCN_E_INVALID
    assert L.ocn_ensemble_step(None, 1) == ocn.OCN_E_INVALID
    assert L.ocn_ensemble_set_tiles(None, 4, 2, 0) == ocn.OCN_E_INVALID


def test_ensemble_members_recipe():
    ms = inputs.ensemble_members(64, seed=0)
    assert len(ms) == 64
    assert all(128 <= m.nx <= 512 and m.nx % 32 == 0 for m in ms)
    assert all(128 <= m.ny <= 256 and m.ny % 32 == 0 for m in ms)
    assert all(32 <= m.nz <= 64 and m.nz % 8 == 0 for m in ms)
    assert all(0.05 <= m.tau0 <= 0.2 and 500 <= m.strat_scale <= 1500 for m in ms)
    total = sum(m.cells for m in ms)
    assert 1.0e8 < total < 3.0e8
    assert ms == inputs.ensemble_members(64, seed=0)
