"""Thin ctypes binding of libocn.so (the C ABI in include/ocn.h).

Argument marshalling only: every step of the ocean path runs in the library's
HIP kernels. PyTorch supplies the device arena (a uint8 tensor) and the HIP
stream; nothing else. Importing this module never falls back to anything: a
missing library raises.
"""
from __future__ import annotations

import ctypes as C
import json
import math
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
          "w": 9, "gu_prev": 10, "gv_prev": 11, "gt_prev": 12, "taux": 13, "tauy": 14, "tstar": 15, "tref": 16,
          "kappa": 17, "visc": 18, "u_pred": 19, "v_pred": 20, "T_pred": 21, "gU_slow": 22, "gV_slow": 23,
          "S": 24, "gs_prev": 25, "sstar": 26, "S_pred": 27, "sref": 28}
FIELDS_3D = {"u", "v", "T", "gu_prev", "gv_prev", "gt_prev", "kappa", "visc", "u_pred", "v_pred", "T_pred",
             "S", "gs_prev", "S_pred"}
# stages of a step (ocn_stage)
STAGE_MIXING, STAGE_TENDENCY, STAGE_BAROTROPIC, STAGE_COLUMN = 0, 1, 2, 3
# Richardson-number mixing constants (Pacanowski and Philander 1981 form)
RI_DEFAULTS = {"nu0": 1e-2, "alpha": 5.0, "nu_b": 1e-4, "kappa_b": 1e-5, "conv": 1.0}

# Functions declared in include/ocn.h.
ABI_FUNCTIONS = ["ocn_abi_version", "ocn_last_error", "ocn_grid_create", "ocn_grid_destroy",
                 "ocn_state_arena_bytes", "ocn_state_init", "ocn_state_destroy", "ocn_set_field",
                 "ocn_get_field", "ocn_set_first_step", "ocn_get_first_step", "ocn_step", "ocn_step_graph",
                 "ocn_diagnostics", "ocn_synchronize", "ocn_stage_timing", "ocn_stage_times",
                 "ocn_checkpoint_bytes", "ocn_checkpoint_save", "ocn_checkpoint_load",
                 "ocn_ensemble_arena_bytes", "ocn_ensemble_init", "ocn_ensemble_destroy", "ocn_ensemble_member",
                 "ocn_ensemble_step", "ocn_ensemble_set_tiles", "ocn_ensemble_autotune",
                 "ocn_mlp_arena_bytes", "ocn_mlp_init", "ocn_mlp_destroy", "ocn_mlp_param_count",
                 "ocn_mlp_set_params", "ocn_mlp_get_params", "ocn_mlp_forward", "ocn_mlp_gradients",
                 "ocn_mlp_train_step", "ocn_closure_workspace_bytes", "ocn_closure_attach",
                 "ocn_closure_detach", "ocn_closure_features", "ocn_closure_kappa", "ocn_closure_convective",
                 "ocn_closure_richardson", "ocn_debug_run_stage", "ocn_diagnostics_noalloc"]


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
                ("salinity", C.c_int32), ("dt", C.c_double), ("chi", C.c_double), ("g", C.c_double),
                ("alpha", C.c_double), ("rho0", C.c_double), ("t_ref", C.c_double), ("kappa", C.c_double),
                ("restore_tau", C.c_double), ("pgf_weight", C.c_double), ("eos", C.c_double * 9),
                ("momentum_form", C.c_int32), ("reserved2", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("tracer_content", C.c_double),
                ("volume", C.c_double), ("volume_mean", C.c_double), ("kinetic_energy", C.c_double),
                ("max_abs_u", C.c_double), ("max_abs_v", C.c_double), ("max_abs_w", C.c_double),
                ("t_min", C.c_double), ("t_max", C.c_double), ("eta_min", C.c_double), ("eta_max", C.c_double),
                ("cfl_adv", C.c_double), ("wet_area", C.c_double), ("nonfinite", C.c_int64),
                ("cfl_bt", C.c_double), ("salt_content", C.c_double)]


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
        L.ocn_debug_run_stage.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_step_graph.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_diagnostics.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.ocn_diagnostics_noalloc.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.ocn_synchronize.argtypes = [C.c_void_p]
        L.ocn_checkpoint_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.ocn_checkpoint_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.ocn_checkpoint_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.ocn_ensemble_arena_bytes.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Params),
                                               C.POINTER(C.c_size_t)]
        L.ocn_ensemble_init.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Params), C.c_void_p, C.c_size_t,
                                        C.c_void_p, C.POINTER(C.c_void_p)]
        L.ocn_ensemble_destroy.argtypes = [C.c_void_p]
        L.ocn_ensemble_member.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]
        L.ocn_ensemble_step.argtypes = [C.c_void_p, C.c_int32]
        L.ocn_ensemble_set_tiles.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        L.ocn_ensemble_autotune.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.ocn_stage_timing.argtypes = [C.c_void_p, C.c_int32]
        _F = C.POINTER(C.c_float)
        L.ocn_mlp_arena_bytes.argtypes = [C.c_int32] * 5 + [C.POINTER(C.c_size_t)]
        L.ocn_mlp_init.argtypes = [C.c_int32] * 5 + [C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.ocn_mlp_destroy.argtypes = [C.c_void_p]
        L.ocn_mlp_param_count.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.ocn_mlp_set_params.argtypes = [C.c_void_p, _F, C.c_size_t]
        L.ocn_mlp_get_params.argtypes = [C.c_void_p, _F, C.c_size_t]
        L.ocn_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.ocn_mlp_gradients.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, _F, C.c_size_t, _F]
        L.ocn_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, _F]
        L.ocn_closure_workspace_bytes.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]
        L.ocn_closure_attach.argtypes = [C.c_void_p, C.c_void_p, _F, C.c_size_t, C.c_void_p, C.c_size_t]
        L.ocn_closure_detach.argtypes = [C.c_void_p]
        L.ocn_closure_convective.argtypes = [C.c_void_p, C.c_double]
        L.ocn_closure_richardson.argtypes = [C.c_void_p] + [C.c_double] * 5
        L.ocn_closure_features.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.ocn_closure_kappa.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
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
    p.pgf_weight = w.pgf_weight
    p.salinity = 1 if getattr(w, "salinity", False) else 0
    p.momentum_form = {"flux": 0, "vector_invariant": 1}[getattr(w, "momentum_form", "flux")]
    if p.salinity:
        for q, c in enumerate(w.eos):
            p.eos[q] = c
    return p


class Grid:
    def __init__(self, w, dz, kbottom):
        desc, self._keep = grid_desc(w, dz, kbottom)
        h = C.c_void_p()
        _check(lib().ocn_grid_create(C.byref(desc), C.byref(h)), "ocn_grid_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ocn_grid_destroy(self.handle)
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
        if self._params.salinity:
            for name in ("S0", "sstar"):
                if name in inp:
                    self.set("S" if name == "S0" else name, inp[name])

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ocn_state_destroy(self.handle)
        self.handle = None

    __del__ = close

    def _shape(self, name):
        if name == "w":
            return (self.nz + 1, self.ny, self.nx)
        if name in ("tref", "sref"):
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

    def step(self, n: int = 1, graph: bool = False):
        """Enqueue n steps; graph=True replays one captured step (needs a non-default stream)."""
        if graph:
            _check(lib().ocn_step_graph(self.handle, int(n)), "ocn_step_graph")
        else:
            _check(lib().ocn_step(self.handle, int(n)), "ocn_step")

    def run_stage(self, stage: int):
        """Enqueue one stage of a step (STAGE_*); no step count, time or start-flag change."""
        _check(lib().ocn_debug_run_stage(self.handle, int(stage)), "ocn_debug_run_stage")

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
        """Accumulated per-stage milliseconds and step count; clears them."""
        ms = np.zeros(4)
        n = C.c_int64()
        _check(lib().ocn_stage_times(self.handle, ms.ctypes.data_as(_D), 4, C.byref(n)), "ocn_stage_times")
        return {"tendency": ms[0], "barotropic": ms[1], "column": ms[2], "closure": ms[3]}, int(n.value)

    def attach_closure(self, net: Optional["Mlp"] = None, norm: Optional[np.ndarray] = None):
        """Use a per-face diffusivity: a prescribed field (net None; set it with set("kappa", ...))
        or the network net, normalising its inputs with norm = [means (din), stds (din)]."""
        import torch
        n = C.c_size_t()
        nh = net._h if net is not None else None
        _check(lib().ocn_closure_workspace_bytes(self.handle, nh, C.byref(n)), "ocn_closure_workspace_bytes")
        self._closure_ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._closure_ws.data_ptr() + 255) // 256 * 256
        if net is not None:
            self._norm = np.ascontiguousarray(norm, dtype=np.float32)
            nptr, ncount = self._norm.ctypes.data_as(C.POINTER(C.c_float)), self._norm.size
        else:
            nptr, ncount = None, 0
        self._closure_net = net
        _check(lib().ocn_closure_attach(self.handle, nh, nptr, ncount, C.c_void_p(aligned), n.value),
               "ocn_closure_attach")

    def set_convective(self, kappa_conv: float):
        """Convective adjustment (needs attach_closure() without a network): kappa_conv where N^2 < 0."""
        _check(lib().ocn_closure_convective(self.handle, float(kappa_conv)), "ocn_closure_convective")

    def set_richardson(self, nu0=RI_DEFAULTS["nu0"], alpha=RI_DEFAULTS["alpha"], nu_b=RI_DEFAULTS["nu_b"],
                       kappa_b=RI_DEFAULTS["kappa_b"], conv=RI_DEFAULTS["conv"]):
        """Richardson-number mixing (needs attach_closure() without a network); nu0 <= 0 turns it off."""
        _check(lib().ocn_closure_richardson(self.handle, float(nu0), float(alpha), float(nu_b), float(kappa_b),
                                            float(conv)), "ocn_closure_richardson")

    def detach_closure(self):
        _check(lib().ocn_closure_detach(self.handle), "ocn_closure_detach")
        self._closure_net = None

    def closure_features(self, din: int, norm: Optional[np.ndarray] = None):
        """Network inputs of every column as a device FP32 tensor [(ny*nx), din]."""
        import torch
        x = torch.empty(self.nx * self.ny, din, dtype=torch.float32, device=self.device)
        nd = None
        if norm is not None:
            nd = torch.from_numpy(np.ascontiguousarray(norm, dtype=np.float32)).to(self.device)
        _check(lib().ocn_closure_features(self.handle, din, C.c_void_p(nd.data_ptr()) if nd is not None else None,
                                          C.c_void_p(x.data_ptr())), "ocn_closure_features")
        self.synchronize()
        return x

    def closure_kappa(self, y):
        """Map network outputs (device FP32 [(ny*nx), ldy >= nz]) to the attached face field."""
        assert y.dtype.is_floating_point and y.is_contiguous()
        _check(lib().ocn_closure_kappa(self.handle, C.c_void_p(y.data_ptr()), y.shape[1]), "ocn_closure_kappa")
        self.synchronize()

    def synchronize(self):
        _check(lib().ocn_synchronize(self.handle), "ocn_synchronize")

    def diagnostics(self, allow_unstable: bool = False) -> dict:
        d = Diag()
        rc = lib().ocn_diagnostics(self.handle, C.byref(d))
        if not (rc == OCN_E_UNSTABLE and allow_unstable):
            _check(rc, "ocn_diagnostics")
        return {name: getattr(d, name) for name, _ in Diag._fields_}


class _Member(Model):
    """A borrowed member state of an ensemble: the state calls of Model, no ownership."""

    def __init__(self, ens, m, w):
        self.w = w
        self.precision = ens.precision
        self.nx, self.ny, self.nz = w.nx, w.ny, w.nz
        h = C.c_void_p()
        _check(lib().ocn_ensemble_member(ens.handle, m, C.byref(h)), "ocn_ensemble_member")
        self.handle = h
        self._ens = ens

    def close(self):
        self.handle = None

    __del__ = close

    def step(self, n: int = 1):
        raise RuntimeError("members advance through Ensemble.step")


def tuning_key(precision: str, workloads) -> str:
    """The autotune cache key of an ensemble: kernel family, precision,
    deepest member, size class (log2 of its cells, rounded) and member count."""
    ws = list(workloads)
    nz = max(w.nz for w in ws)
    size_class = int(round(math.log2(max(sum(w.cells for w in ws), 1))))
    return f"ensemble/{precision}/nz{nz}/cells2^{size_class}/members{len(ws)}"


def autotune_cache_load(path: str) -> dict:
    """Autotuned choices stored in a JSON file (empty if it does not exist or
    does not hold a JSON object: the tuner then times the choices again and
    the next store rewrites the file)."""
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (FileNotFoundError, ValueError):
        return {}


def autotune_cache_store(path: str, key: str, rec: dict):
    """Add (or replace) one choice in the cache file, written atomically."""
    data = autotune_cache_load(path)
    data[key] = rec
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class Ensemble:
    """Independent basins stepped together: one tendency launch and one column
    launch per step for all members, barotropic launches per substep group, the
    step replayed from a HIP graph on a dedicated stream."""

    def __init__(self, workloads, precision: str = "fp32", inputs_list=None, device: str = "cuda:0",
                 baro_fuse: int = 0):
        import torch

        self.precision = precision
        self.workloads = list(workloads)
        if inputs_list is None:
            inputs_list = [_inputs.make_inputs(w) for w in self.workloads]
        p0 = self.workloads[0]
        for w in self.workloads:
            if (w.dt, w.n_substeps, w.kappa, w.chi, w.pgf_weight, w.g, w.alpha, w.rho0, w.t_ref, w.restore_days) != \
                    (p0.dt, p0.n_substeps, p0.kappa, p0.chi, p0.pgf_weight, p0.g, p0.alpha, p0.rho0, p0.t_ref,
                     p0.restore_days):
                raise ValueError("ensemble members must share time step and physical parameters")
        self.grids = [Grid(w, inp["dz"], inp["kbottom"]) for w, inp in zip(self.workloads, inputs_list)]
        self._params = params(p0, precision, baro_fuse)
        n = len(self.grids)
        arr = (C.c_void_p * n)(*[g.handle.value for g in self.grids])
        nbytes = C.c_size_t()
        _check(lib().ocn_ensemble_arena_bytes(arr, n, C.byref(self._params), C.byref(nbytes)),
               "ocn_ensemble_arena_bytes")
        self.device = torch.device(device)
        self.arena = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.arena.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.Stream(self.device)   # graph capture needs a non-default stream
        h = C.c_void_p()
        _check(lib().ocn_ensemble_init(arr, n, C.byref(self._params), C.c_void_p(aligned), C.c_size_t(nbytes.value),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)), "ocn_ensemble_init")
        self.handle = h
        self.members = [_Member(self, m, w) for m, w in enumerate(self.workloads)]
        for mem, inp in zip(self.members, inputs_list):
            for name in ("T0", "taux", "tauy", "tstar"):
                if name in inp:
                    mem.set("T" if name == "T0" else name, inp[name])

    def close(self):
        if getattr(self, "handle", None):
            for mem in self.members:
                mem.close()
            lib().ocn_ensemble_destroy(self.handle)
            self.handle = None

    __del__ = close

    def step(self, n: int = 1):
        _check(lib().ocn_ensemble_step(self.handle, int(n)), "ocn_ensemble_step")

    def synchronize(self):
        self.stream.synchronize()

    def set_tiles(self, tend_rows: int = 0, baro_fuse: int = 0, persistent: int = 0):
        _check(lib().ocn_ensemble_set_tiles(self.handle, int(tend_rows), int(baro_fuse), int(persistent)),
               "ocn_ensemble_set_tiles")

    def tuning_key(self) -> str:
        return tuning_key(self.precision, self.workloads)

    def autotune(self, trial_steps: int = 3, cache: Optional[str] = None) -> dict:
        """Time every choice and keep the fastest. With a cache file (JSON), a
        choice stored under tuning_key() is applied without timing, and a new
        one is stored."""
        key = self.tuning_key()
        if cache is not None:
            hit = autotune_cache_load(cache).get(key)
            if isinstance(hit, dict) and all(isinstance(hit.get(k), int) for k in ("tend_rows", "baro_fuse")):
                self.set_tiles(hit["tend_rows"], hit["baro_fuse"], hit.get("persistent", 0))
                return dict(hit, cached=True)
        r, f, p, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().ocn_ensemble_autotune(self.handle, int(trial_steps), C.byref(r), C.byref(f), C.byref(p),
                                           C.byref(ms)), "ocn_ensemble_autotune")
        rec = {"tend_rows": r.value, "baro_fuse": f.value, "persistent": p.value, "ms_per_step": ms.value}
        if cache is not None:
            autotune_cache_store(cache, key, rec)
        return dict(rec, cached=False)

    @property
    def cells(self) -> int:
        return sum(w.cells for w in self.workloads)


class Mlp:
    """The closure network (Linear-ReLU-Linear-ReLU-Linear) on the GPU's matrix
    cores: BF16 products with FP32 accumulation, FP32 master weights and Adam.

    Parameters travel as one packed FP32 vector: W1 (din x h1, row-major), b1,
    W2 (h1 x h2), b2, W3 (h2 x dout), b3. Batches are FP32 torch tensors on the
    device, rows x din in and rows x dout out.
    """

    def __init__(self, din: int, h1: int, h2: int, dout: int, max_batch: int, device: str = "cuda:0"):
        import torch
        L = lib()
        self.shape = (din, h1, h2, dout)
        self.max_batch = max_batch
        self.device = torch.device(device)
        nbytes = C.c_size_t()
        _check(L.ocn_mlp_arena_bytes(din, h1, h2, dout, max_batch, C.byref(nbytes)), "ocn_mlp_arena_bytes")
        self._arena = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self._arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.ocn_mlp_init(din, h1, h2, dout, max_batch, C.c_void_p(aligned), nbytes.value,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h)), "ocn_mlp_init")
        self._h = h
        n = C.c_size_t()
        _check(L.ocn_mlp_param_count(h, C.byref(n)), "ocn_mlp_param_count")
        self.nparam = n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ocn_mlp_destroy(h)
            self._h = None

    def unpack(self, flat: np.ndarray):
        din, h1, h2, dout = self.shape
        sizes = [(din, h1), (h1,), (h1, h2), (h2,), (h2, dout), (dout,)]
        out, o = [], 0
        for sz in sizes:
            n = int(np.prod(sz))
            out.append(flat[o:o + n].reshape(sz))
            o += n
        return out

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.nparam
        _check(lib().ocn_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "ocn_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparam, dtype=np.float32)
        _check(lib().ocn_mlp_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "ocn_mlp_get_params")
        return a

    def _dev(self, x, cols):
        import torch
        assert x.dtype == torch.float32 and x.is_contiguous() and x.device == self.device
        assert x.dim() == 2 and x.shape[1] == cols and 1 <= x.shape[0] <= self.max_batch
        return x.shape[0]

    def forward(self, x):
        import torch
        rows = self._dev(x, self.shape[0])
        y = torch.empty(rows, self.shape[3], dtype=torch.float32, device=self.device)
        _check(lib().ocn_mlp_forward(self._h, C.c_void_p(x.data_ptr()), rows, C.c_void_p(y.data_ptr())),
               "ocn_mlp_forward")
        return y

    def gradients(self, x, t):
        rows = self._dev(x, self.shape[0])
        assert self._dev(t, self.shape[3]) == rows
        g = np.empty(self.nparam, dtype=np.float32)
        loss = C.c_float()
        _check(lib().ocn_mlp_gradients(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), rows,
                                       g.ctypes.data_as(C.POINTER(C.c_float)), g.size, C.byref(loss)),
               "ocn_mlp_gradients")
        return float(loss.value), g

    def train_step(self, x, t, lr: float, want_loss: bool = True):
        rows = self._dev(x, self.shape[0])
        assert self._dev(t, self.shape[3]) == rows
        loss = C.c_float()
        _check(lib().ocn_mlp_train_step(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), rows,
                                        float(lr), C.byref(loss) if want_loss else None),
               "ocn_mlp_train_step")
        return float(loss.value) if want_loss else None
