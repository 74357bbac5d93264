"""Thin ctypes binding of libocn.so (the C ABI in include/ocn.h).

Argument marshalling only: every step of the ocean path runs in the library's
HIP kernels. PyTorch supplies the device arena (a uint8 tensor) and the HIP
stream; nothing else. Importing this module never falls back to anything: a
missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import inputs as _inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocn.so")

OCN_OK, OCN_E_INVALID, OCN_E_NOMEM, OCN_E_DEVICE, OCN_E_UNSTABLE, OCN_E_STATE, OCN_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
OCN_FP64, OCN_FP32 = 0, 1
OCN_CARTESIAN, OCN_LATLON = 0, 1

FIELDS = {"u": 0, "v": 1, "T": 2, "eta": 3, "U": 4, "V": 5, "eta_mean": 6, "U_mean": 7, "V_mean": 8,
          "w": 9, "gu_prev": 10, "gv_prev": 11, "gt_prev": 12, "taux": 13, "tauy": 14, "tstar": 15, "tref": 16}
FIELDS_3D = {"u", "v", "T", "gu_prev", "gv_prev", "gt_prev"}

# Functions declared in include/ocn.h.
ABI_FUNCTIONS = ["ocn_abi_version", "ocn_last_error", "ocn_grid_create", "ocn_grid_destroy",
                 "ocn_state_arena_bytes", "ocn_state_init", "ocn_state_destroy", "ocn_set_field",
                 "ocn_get_field", "ocn_set_first_step", "ocn_get_first_step", "ocn_step",
                 "ocn_diagnostics", "ocn_synchronize", "ocn_stage_timing", "ocn_stage_times",
                 "ocn_checkpoint_bytes", "ocn_checkpoint_save", "ocn_checkpoint_load"]


class OcnError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("halo", C.c_int32),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32), ("coords", C.c_int32), ("reserved", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("f0", C.c_double), ("beta", C.c_double), ("radius", C.c_double), ("omega", C.c_double),
                ("dz", C.POINTER(C.c_double)), ("kbottom", C.POINTER(C.c_int32))]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_substeps", C.c_int32), ("baro_fuse", C.c_int32),
                ("reserved1", C.c_int32), ("dt", C.c_double), ("chi", C.c_double), ("g", C.c_double),
                ("alpha", C.c_double), ("rho0", C.c_double), ("t_ref", C.c_double), ("kappa", C.c_double),
                ("restore_tau", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("tracer_content", C.c_double),
                ("volume", C.c_double), ("volume_mean", C.c_double), ("kinetic_energy", C.c_double),
                ("max_abs_u", C.c_double), ("max_abs_v", C.c_double), ("max_abs_w", C.c_double),
                ("t_min", C.c_double), ("t_max", C.c_double), ("eta_min", C.c_double), ("eta_max", C.c_double),
                ("cfl_adv", C.c_double), ("wet_area", C.c_double), ("nonfinite", C.c_int64)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    """Load libocn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2309_06662_amd.build")
        L = C.CDLL(LIB_PATH)
        L.ocn_abi_version.restype = C.c_uint32
        L.ocn_last_error.restype = C.c_char_p
        L.ocn_grid_create.argtypes = [C.POINTER(GridDesc), C.POINTER(C.c_void_p)]
        L.ocn_grid_destroy.argtypes = [C.c_void_p]
        L.ocn_state_arena_bytes.argtypes = [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_size_t)]
        L.ocn_state_init.argtypes = [C.c_void_p, C.POINTER(Params), C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.POINTER(C.c_void_p)]
        L.ocn_state_destroy.argtypes = [C.c_void_p]
        L.ocn_set_field.argtypes = [C.c_void_p, C.c_int32, _D, C.c_size_t]
        L.ocn_get_field.argtypes = [C.c_void_p, C.c_int32, _D, C.c_size_t]
        L.ocn_set_first_step.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_get_first_step.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.ocn_step.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_diagnostics.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.ocn_synchronize.argtypes = [C.c_void_p]
        L.ocn_checkpoint_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.ocn_checkpoint_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.ocn_checkpoint_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.ocn_stage_timing.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_stage_times.argtypes = [C.c_void_p, _D, C.c_int32, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != OCN_OK:
        raise OcnError(rc, where, lib().ocn_last_error().decode(errors="replace"))


def grid_desc(w: "_inputs.Workload", dz: np.ndarray, kbottom: Optional[np.ndarray]):
    """Fill an ocn_grid_desc from a workload; returns (desc, keep-alive arrays)."""
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    kb = None if kbottom is None else np.ascontiguousarray(kbottom, dtype=np.int32)
    d = GridDesc()
    d.nx, d.ny, d.nz, d.halo = w.nx, w.ny, w.nz, w.halo
    d.periodic_x, d.periodic_y = int(w.periodic_x), int(w.periodic_y)
    d.coords = OCN_LATLON if w.coords == "latlon" else OCN_CARTESIAN
    d.reserved = 0
    d.x0, d.y0, d.dx, d.dy = w.x0, w.y0, w.dx, w.dy
    d.f0, d.beta, d.radius, d.omega = w.f0, w.beta, w.radius, w.omega
    d.dz = dz.ctypes.data_as(_D)
    d.kbottom = kb.ctypes.data_as(C.POINTER(C.c_int32)) if kb is not None else C.POINTER(C.c_int32)()
    return d, (dz, kb)


def params(w: "_inputs.Workload", precision: str, baro_fuse: int = 0) -> Params:
    p = Params()
    p.precision = OCN_FP32 if precision == "fp32" else OCN_FP64
    p.n_substeps = w.n_substeps
    p.baro_fuse = baro_fuse
    p.dt, p.chi, p.g, p.alpha, p.rho0, p.t_ref, p.kappa = w.dt, w.chi, w.g, w.alpha, w.rho0, w.t_ref, w.kappa
    p.restore_tau = w.restore_days * 86400.0 if w.restore_days > 0 else 0.0
    return p


class Grid:
    def __init__(self, w, dz, kbottom):
        desc, self._keep = grid_desc(w, dz, kbottom)
        h = C.c_void_p()
        _check(lib().ocn_grid_create(C.byref(desc), C.byref(h)), "ocn_grid_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().ocn_grid_destroy(self.handle)
            self.handle = None

    __del__ = close


class Model:
    """One ocean state on a GPU. Fields are float64 numpy arrays: 3D [nz, ny, nx], 2D [ny, nx]."""

    def __init__(self, w, precision: str = "fp64", inp: Optional[Dict[str, np.ndarray]] = None,
                 device: str = "cuda:0", stream=None, baro_fuse: int = 0):
        import torch  # device memory and the stream only

        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        self.w = w
        self.precision = precision
        self.nx, self.ny, self.nz = w.nx, w.ny, w.nz
        if inp is None:
            inp = _inputs.make_inputs(w)
        self.grid = Grid(w, inp["dz"], inp["kbottom"])
        self._params = params(w, precision, baro_fuse)
        nbytes = C.c_size_t()
        _check(lib().ocn_state_arena_bytes(self.grid.handle, C.byref(self._params), C.byref(nbytes)),
               "ocn_state_arena_bytes")
        self.device = torch.device(device)
        self.arena = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().ocn_state_init(self.grid.handle, C.byref(self._params), C.c_void_p(aligned),
                                    C.c_size_t(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "ocn_state_init")
        self.handle = h
        for name in ("T0", "taux", "tauy", "tstar"):
            if name in inp:
                self.set("T" if name == "T0" else name, inp[name])

    def close(self):
        if getattr(self, "handle", None):
            lib().ocn_state_destroy(self.handle)
            self.handle = None

    __del__ = close

    def _shape(self, name):
        if name == "w":
            return (self.nz + 1, self.ny, self.nx)
        if name == "tref":
            return (self.nz,)
        return (self.nz, self.ny, self.nx) if name in FIELDS_3D else (self.ny, self.nx)

    def set(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self._shape(name))
        _check(lib().ocn_set_field(self.handle, FIELDS[name], a.ctypes.data_as(_D), a.size), f"set {name}")

    def get(self, name: str) -> np.ndarray:
        out = np.empty(self._shape(name), dtype=np.float64)
        _check(lib().ocn_get_field(self.handle, FIELDS[name], out.ctypes.data_as(_D), out.size), f"get {name}")
        return out

    @property
    def first_step(self) -> bool:
        f = C.c_int32()
        _check(lib().ocn_get_first_step(self.handle, C.byref(f)), "ocn_get_first_step")
        return bool(f.value)

    @first_step.setter
    def first_step(self, v: bool):
        _check(lib().ocn_set_first_step(self.handle, int(bool(v))), "ocn_set_first_step")

    def step(self, n: int = 1):
        _check(lib().ocn_step(self.handle, int(n)), "ocn_step")

    def checkpoint(self) -> bytes:
        n = C.c_size_t()
        _check(lib().ocn_checkpoint_bytes(self.handle, C.byref(n)), "ocn_checkpoint_bytes")
        buf = C.create_string_buffer(n.value)
        _check(lib().ocn_checkpoint_save(self.handle, buf, n.value), "ocn_checkpoint_save")
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().ocn_checkpoint_load(self.handle, buf, len(blob)), "ocn_checkpoint_load")

    def stage_timing(self, enable: bool):
        _check(lib().ocn_stage_timing(self.handle, int(bool(enable))), "ocn_stage_timing")

    def stage_times(self):
        """Accumulated (tendency, barotropic, column) milliseconds and step count; clears them."""
        ms = np.zeros(3)
        n = C.c_int64()
        _check(lib().ocn_stage_times(self.handle, ms.ctypes.data_as(_D), 3, C.byref(n)), "ocn_stage_times")
        return {"tendency": ms[0], "barotropic": ms[1], "column": ms[2]}, int(n.value)

    def synchronize(self):
        _check(lib().ocn_synchronize(self.handle), "ocn_synchronize")

    def diagnostics(self, allow_unstable: bool = False) -> dict:
        d = Diag()
        rc = lib().ocn_diagnostics(self.handle, C.byref(d))
        if not (rc == OCN_E_UNSTABLE and allow_unstable):
            _check(rc, "ocn_diagnostics")
        return {name: getattr(d, name) for name, _ in Diag._fields_}
