"""ctypes loader for the plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ORC_U, ORC_V, ORC_T, ORC_ETA, ORC_UBT, ORC_VBT = 0, 1, 2, 3, 4, 5
ORC_ETA_MEAN, ORC_UBT_MEAN, ORC_VBT_MEAN, ORC_W = 6, 7, 8, 9
ORC_GU_PREV, ORC_GV_PREV, ORC_GT_PREV = 10, 11, 12
ORC_TAUX, ORC_TAUY, ORC_TSTAR, ORC_P, ORC_KAPPA, ORC_VISC = 13, 14, 15, 16, 17, 18
TERM_ADV, TERM_COR, TERM_PGF, TERM_WIND, TERM_RESTORE, TERM_ALL = 1, 2, 4, 8, 16, 31
NDIAG = 18
DIAG_NAMES = ["step", "time", "tracer_content", "volume", "volume_mean", "kinetic_energy",
              "max_abs_u", "max_abs_v", "max_abs_w", "t_min", "t_max", "eta_min", "eta_max",
              "nonfinite", "cfl_adv", "wet_area", "cfl_bt", "salt_content"]
STAGE_MIXING, STAGE_TENDENCY, STAGE_BAROTROPIC, STAGE_COLUMN = 0, 1, 2, 3

FIELD_IDS = {"u": ORC_U, "v": ORC_V, "T": ORC_T, "eta": ORC_ETA, "U": ORC_UBT, "V": ORC_VBT,
             "eta_mean": ORC_ETA_MEAN, "U_mean": ORC_UBT_MEAN, "V_mean": ORC_VBT_MEAN,
             "w": ORC_W, "gu_prev": ORC_GU_PREV, "gv_prev": ORC_GV_PREV, "gt_prev": ORC_GT_PREV,
             "taux": ORC_TAUX, "tauy": ORC_TAUY, "tstar": ORC_TSTAR, "p": ORC_P, "kappa": ORC_KAPPA,
             "visc": ORC_VISC, "u_pred": 19, "v_pred": 20, "T_pred": 21, "gU_slow": 22, "gV_slow": 23,
             "S": 24, "gs_prev": 25, "sstar": 26, "S_pred": 27}
FIELDS_3D = {"u", "v", "T", "gu_prev", "gv_prev", "gt_prev", "p", "kappa", "visc", "u_pred", "v_pred", "T_pred",
             "S", "gs_prev", "S_pred"}
# Richardson-number mixing constants of the reading (Pacanowski and Philander 1981 form)
RI_DEFAULTS = {"nu0": 1e-2, "alpha": 5.0, "nu_b": 1e-4, "kappa_b": 1e-5, "conv": 1.0}


# momentum advection forms (orc_desc.momentum_form)
MOMENTUM_FORMS = {"flux": 0, "vector_invariant": 1}


class OrcDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32), ("coords", C.c_int32),
                ("n_substeps", C.c_int32), ("salinity", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("f0", C.c_double), ("beta", C.c_double), ("radius", C.c_double), ("omega", C.c_double),
                ("dt", C.c_double), ("chi", C.c_double), ("g", C.c_double), ("alpha", C.c_double),
                ("rho0", C.c_double), ("t_ref", C.c_double), ("kappa", C.c_double),
                ("restore_tau", C.c_double), ("pgf_weight", C.c_double),
                ("eos_a0", C.c_double), ("eos_b0", C.c_double), ("eos_lambda1", C.c_double),
                ("eos_lambda2", C.c_double), ("eos_mu1", C.c_double), ("eos_mu2", C.c_double),
                ("eos_nu", C.c_double), ("eos_t0", C.c_double), ("eos_s0", C.c_double),
                ("momentum_form", C.c_int32), ("reserved", C.c_int32)]


_lib = None
_P = np.ctypeslib.ndpointer
_D = C.POINTER(C.c_double)


def lib():
    """Load liboracle.so, building it with gcc first if it is missing or stale
    (the -O3 build of the same sources when OCN_ORACLE_BUILD=o3, for timing)."""
    global _lib
    if _lib is None:
        variant = "o3" if os.environ.get("OCN_ORACLE_BUILD") == "o3" else "o2"
        path = _build.lib_path(variant)
        if (not os.path.exists(path)) or os.path.getmtime(path) < max(
                [os.path.getmtime(f) for f in _build.SRCS] + [os.path.getmtime(os.path.join(_build.HERE, "ocean_oracle.h"))]):
            _build.build(variant=variant)
        L = C.CDLL(path)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcDesc), _D, C.POINTER(C.c_int32)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int, _D]
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int, _D]
        L.orc_set_first_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_first_step.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_run_stage.argtypes = [C.c_void_p, C.c_int]
        L.orc_diagnostics.argtypes = [C.c_void_p, _D]
        L.orc_eval_tendencies.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D]
        L.orc_buoyancy.restype = C.c_double
        L.orc_buoyancy.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        for name in ("orc_weno5z",):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 5
        L.orc_weno3.restype = C.c_double
        L.orc_weno3.argtypes = [C.c_double] * 3
        L.orc_reconstruct.restype = C.c_double
        L.orc_reconstruct.argtypes = [_D, C.POINTER(C.c_int32)]
        L.orc_thomas.argtypes = [C.c_int, _D, _D, _D, _D, _D]
        L.orc_neumaier_sum.restype = C.c_double
        L.orc_neumaier_sum.argtypes = [_D, C.c_int64]
        L.orc_column_zflux.argtypes = [C.c_int, _D, C.POINTER(C.c_int32), _D, _D]
        L.orc_set_convective.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_richardson.argtypes = [C.c_void_p] + [C.c_double] * 5
        L.orc_closure_features.argtypes = [C.c_void_p, C.c_int, _D, _D, _D]
        L.orc_closure_kappa.argtypes = [C.c_void_p, _D, C.c_double, _D]
        L.orc_mlp_forward.argtypes = [_D, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int] + [_D] * 9
        L.orc_mlp_backward.restype = C.c_double
        L.orc_mlp_backward.argtypes = [_D, _D, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int] + [_D] * 12
        L.orc_adam.argtypes = [_D, _D, _D, _D, C.c_int64, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def desc_from_workload(w) -> OrcDesc:
    d = OrcDesc()
    d.nx, d.ny, d.nz = w.nx, w.ny, w.nz
    d.periodic_x, d.periodic_y = int(w.periodic_x), int(w.periodic_y)
    d.coords = 1 if w.coords == "latlon" else 0
    d.n_substeps = w.n_substeps
    d.x0, d.y0, d.dx, d.dy = w.x0, w.y0, w.dx, w.dy
    d.f0, d.beta, d.radius, d.omega = w.f0, w.beta, w.radius, w.omega
    d.dt, d.chi, d.g, d.alpha, d.rho0, d.t_ref = w.dt, w.chi, w.g, w.alpha, w.rho0, w.t_ref
    d.kappa = w.kappa
    d.restore_tau = w.restore_days * 86400.0 if w.restore_days > 0 else 0.0
    d.pgf_weight = w.pgf_weight
    d.salinity = int(w.salinity)
    d.momentum_form = MOMENTUM_FORMS[getattr(w, "momentum_form", "flux")]
    (d.eos_a0, d.eos_b0, d.eos_lambda1, d.eos_lambda2, d.eos_mu1, d.eos_mu2, d.eos_nu, d.eos_t0,
     d.eos_s0) = w.eos
    return d


class OracleModel:
    """One oracle ocean state. Fields are numpy float64 arrays, 3D [nz, ny, nx], 2D [ny, nx]."""

    def __init__(self, w, dz: np.ndarray, kbottom: np.ndarray):
        self.w = w
        self.nx, self.ny, self.nz = w.nx, w.ny, w.nz
        self._desc = desc_from_workload(w)
        dz = np.ascontiguousarray(dz, dtype=np.float64)
        kb = np.ascontiguousarray(kbottom, dtype=np.int32)
        h = lib().orc_create(C.byref(self._desc), _dptr(dz), _iptr(kb))
        if not h:
            raise ValueError("orc_create rejected the grid")
        self._h = C.c_void_p(h)

    @classmethod
    def from_inputs(cls, w, inp) -> "OracleModel":
        m = cls(w, inp["dz"], inp["kbottom"])
        m.set("T", inp["T0"])
        m.set("taux", inp["taux"])
        m.set("tauy", inp["tauy"])
        m.set("tstar", inp["tstar"])
        if w.salinity:
            m.set("S", inp["S0"])
            m.set("sstar", inp["sstar"])
        return m

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    __del__ = close

    def _shape(self, name):
        if name == "w":
            return (self.nz + 1, self.ny, self.nx)
        return (self.nz, self.ny, self.nx) if name in FIELDS_3D else (self.ny, self.nx)

    def set(self, name: str, arr: np.ndarray):
        if name == "kappa" and arr is None:  # back to the constant diffusivity
            lib().orc_set_field(self._h, ORC_KAPPA, None)
            return
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self._shape(name))
        if lib().orc_set_field(self._h, FIELD_IDS[name], _dptr(a)) != 0:
            raise ValueError(name)

    def get(self, name: str) -> np.ndarray:
        out = np.empty(self._shape(name), dtype=np.float64)
        if lib().orc_get_field(self._h, FIELD_IDS[name], _dptr(out)) != 0:
            raise ValueError(name)
        return out

    @property
    def first_step(self) -> bool:
        return bool(lib().orc_get_first_step(self._h))

    @first_step.setter
    def first_step(self, v: bool):
        lib().orc_set_first_step(self._h, int(bool(v)))

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def run_stage(self, stage: int):
        """One stage of a step (STAGE_*), without advancing the step count, time or start flag."""
        if lib().orc_run_stage(self._h, int(stage)) != 0:
            raise ValueError(stage)

    def diagnostics(self) -> dict:
        out = np.zeros(NDIAG, dtype=np.float64)
        lib().orc_diagnostics(self._h, _dptr(out))
        return dict(zip(DIAG_NAMES, out.tolist()))

    def set_convective(self, kappa_conv: float):
        """Convective adjustment: kappa_conv on faces with N^2 < 0 at the start of every step (<= 0: off)."""
        lib().orc_set_convective(self._h, float(kappa_conv))

    def set_richardson(self, nu0=RI_DEFAULTS["nu0"], alpha=RI_DEFAULTS["alpha"], nu_b=RI_DEFAULTS["nu_b"],
                       kappa_b=RI_DEFAULTS["kappa_b"], conv=RI_DEFAULTS["conv"]):
        """Richardson-number mixing from the state at the start of every step (nu0 <= 0: off);
        the faces of the current state are diagnosed at once ("kappa", "visc")."""
        lib().orc_set_richardson(self._h, float(nu0), float(alpha), float(nu_b), float(kappa_b), float(conv))

    def closure_features(self, din: int, mean=None, std=None) -> np.ndarray:
        """Per-column network inputs, (ny*nx) x din (feature order in ocean_oracle.c)."""
        mean = np.zeros(din) if mean is None else _c(mean)
        std = np.ones(din) if std is None else _c(std)
        X = np.zeros((self.ny * self.nx, din))
        if lib().orc_closure_features(self._h, din, _dptr(mean), _dptr(std), _dptr(X)) != 0:
            raise ValueError("din must be at least 4 nz + 3")
        return X

    def closure_kappa(self, Y, kappa0: float) -> np.ndarray:
        """Face diffusivity [nz, ny, nx] from network outputs Y ((ny*nx) x nz, log10 kappa on faces, slot 0 unused)."""
        Y = _c(Y).reshape(self.ny * self.nx, self.nz)
        kw = np.zeros((self.nz, self.ny, self.nx))
        lib().orc_closure_kappa(self._h, _dptr(Y), kappa0, _dptr(kw))
        return kw

    def tendencies(self, terms: int = TERM_ALL, salinity: bool = False):
        """(gu, gv, gt), or (gu, gv, gt, gs) with salinity=True."""
        shape = (self.nz, self.ny, self.nx)
        gu, gv, gt, gs = (np.zeros(shape) for _ in range(4))
        lib().orc_eval_tendencies(self._h, terms, _dptr(gu), _dptr(gv), _dptr(gt), _dptr(gs))
        return (gu, gv, gt, gs) if salinity else (gu, gv, gt)

    def buoyancy(self, T: float, S: float, z: float) -> float:
        """b = -g rho'/rho0 of water (T, S) at depth z (m) under the model's equation of state."""
        return lib().orc_buoyancy(self._h, float(T), float(S), float(z))


def weno5z(a, b, c, d, e) -> float:
    return lib().orc_weno5z(a, b, c, d, e)


def weno3(b, c, d) -> float:
    return lib().orc_weno3(b, c, d)


def reconstruct(s, ok) -> float:
    s = np.ascontiguousarray(s, dtype=np.float64)
    ok = np.ascontiguousarray(ok, dtype=np.int32)
    return lib().orc_reconstruct(_dptr(s), _iptr(ok))


def thomas(a, b, c, d) -> np.ndarray:
    a, b, c, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d))
    x = np.zeros_like(d)
    lib().orc_thomas(len(d), _dptr(a), _dptr(b), _dptr(c), _dptr(d), _dptr(x))
    return x


def neumaier_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_neumaier_sum(_dptr(x), len(x))


def column_zflux(phi, wet, wface) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    wet = np.ascontiguousarray(wet, dtype=np.int32)
    wface = np.ascontiguousarray(wface, dtype=np.float64)
    out = np.zeros(len(phi) + 1)
    lib().orc_column_zflux(len(phi), _dptr(phi), _iptr(wet), _dptr(wface), _dptr(out))
    return out


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mlp_forward(X, W1, b1, W2, b2, W3, b3):
    """Network output and hidden activations: (Y, H1, H2)."""
    X, W1, b1, W2, b2, W3, b3 = (_c(a) for a in (X, W1, b1, W2, b2, W3, b3))
    n, din = X.shape
    h1, h2, dout = W1.shape[1], W2.shape[1], W3.shape[1]
    H1, H2, Y = np.zeros((n, h1)), np.zeros((n, h2)), np.zeros((n, dout))
    lib().orc_mlp_forward(_dptr(X), n, din, h1, h2, dout, _dptr(W1), _dptr(b1), _dptr(W2), _dptr(b2), _dptr(W3),
                          _dptr(b3), _dptr(H1), _dptr(H2), _dptr(Y))
    return Y, H1, H2


def mlp_backward(X, T, W1, b1, W2, b2, W3, b3):
    """Mean-squared loss L = sum (Y - T)^2 / (2 n dout) and its gradients (gW1, gb1, gW2, gb2, gW3, gb3)."""
    X, T, W1, b1, W2, b2, W3, b3 = (_c(a) for a in (X, T, W1, b1, W2, b2, W3, b3))
    n, din = X.shape
    h1, h2, dout = W1.shape[1], W2.shape[1], W3.shape[1]
    grads = [np.zeros_like(a) for a in (W1, b1, W2, b2, W3, b3)]
    loss = lib().orc_mlp_backward(_dptr(X), _dptr(T), n, din, h1, h2, dout, _dptr(W1), _dptr(b1), _dptr(W2),
                                  _dptr(b2), _dptr(W3), _dptr(b3), *[_dptr(g) for g in grads])
    return loss, grads


def adam(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays p, m, v with gradient g at step t."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g)
    lib().orc_adam(_dptr(p), _dptr(g), _dptr(m), _dptr(v), p.size, int(t), lr, beta1, beta2, eps)
