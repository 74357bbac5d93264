"""Pins of the oracle's compensated sums and diagnostics (paper Sec. 6 reports
conservation-style integrals and timings; the diagnostics here are the usual
budget quantities of an ocean step).

- Neumaier summation against math.fsum (correctly rounded) on arrays built to
  defeat plain summation: huge cancelling terms around small ones;
- every entry of the diagnostics vector against an independent computation in
  numpy from the state's fields, the wet masks and the row metrics: tracer
  content sum V_c T, free-surface volume sum A_c eta (and of the substep
  average), kinetic energy 1/2 sum (V_u u^2 + V_v v^2), the largest |u|, |v|
  and |w| (w from continuity, integrated up from the bottom), temperature and
  free-surface extrema, the advective and barotropic CFL numbers, the wet
  area and the count of non-finite cells and columns.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, metrics, small_latlon

U = 2.0 ** -53


def test_neumaier_recovers_what_cancellation_hides():
    assert oracle.neumaier_sum([1e100, 1.0, -1e100]) == 1.0
    assert oracle.neumaier_sum([1.0, 1e100, 1.0, -1e100]) == 2.0
    assert oracle.neumaier_sum([3.0, 1e16, -1e16, 2.0 ** -30]) == 3.0 + 2.0 ** -30
    assert oracle.neumaier_sum([]) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_neumaier_against_fsum(seed):
    rng = np.random.default_rng(seed)
    n = 4000
    big = rng.uniform(-1, 1, n // 4) * 10.0 ** rng.integers(10, 18, n // 4)
    small = rng.standard_normal(n // 2)
    x = np.concatenate([big, small, -big])
    rng.shuffle(x)
    exact = math.fsum(x)
    got = oracle.neumaier_sum(x)
    # Neumaier: |s - S| <= 2u|S| + O(n u^2) sum|x|
    bound = 2 * U * abs(exact) + 4 * n * U * U * np.abs(x).sum()
    assert abs(got - exact) <= bound, (got, exact, bound)
    # the plain left-to-right sum misses by far more on the same data
    naive = 0.0
    for v in x:
        naive += v
    assert abs(naive - exact) > 100 * bound


def _continuity_w(w, u, v, wu, wv, dz):
    """Vertical velocity on z-faces from continuity, integrated up from zero at the bottom."""
    _, dxv, dy, area = metrics(w)
    U3 = np.where(wu, u, 0.0) * dy * dz[:, None, None]
    V3 = np.where(wv, v, 0.0) * dxv[None, :-1, None] * dz[:, None, None]
    Ue = np.roll(U3, -1, axis=2) if w.periodic_x else np.concatenate([U3[:, :, 1:], np.zeros_like(U3[:, :, :1])], 2)
    Vn = np.concatenate([V3[:, 1:, :], np.zeros_like(V3[:, :1, :])], 1)
    div = (Ue - U3) + (Vn - V3)
    W = np.zeros((w.nz + 1, w.ny, w.nx))
    for k in range(w.nz):
        W[k + 1] = W[k] - div[k]
    return W / area[None, :, None]


def _expected(w, m, kb, dz, steps):
    wet, wu, wv = masks(w, kb)
    dxc, dxv, dy, area = metrics(w)
    col = kb > 0
    u, v, T = m.get("u"), m.get("v"), m.get("T")
    eta, etam = m.get("eta"), m.get("eta_mean")
    vol_c = area[None, :, None] * dz[:, None, None] * np.ones((1, 1, w.nx))
    vol_v = (dxv[:-1] * dy)[None, :, None] * dz[:, None, None] * np.ones((1, 1, w.nx))
    a2 = area[:, None] * np.ones((1, w.nx))
    wf = _continuity_w(w, u, v, wu, wv, dz)
    k = np.arange(w.nz + 1)[:, None, None]
    face_wet = np.zeros((w.nz + 1, w.ny, w.nx), dtype=bool)
    face_wet[1:w.nz] = wet[:-1] & wet[1:]
    dzc = np.zeros(w.nz + 1)
    dzc[1:w.nz] = 0.5 * (dz[:-1] + dz[1:])
    cfl = max(np.max(np.where(wu, np.abs(u) * w.dt / dxc[None, :, None], 0.0)),
              np.max(np.where(wv, np.abs(v) * w.dt / dy, 0.0)),
              np.max(np.where(face_wet, np.abs(wf) * w.dt / np.where(face_wet, dzc[k], 1.0), 0.0)))
    return {
        "step": float(steps), "time": steps * w.dt,
        "tracer_content": math.fsum((vol_c * T)[wet]),
        "volume": math.fsum((a2 * eta)[col]),
        "volume_mean": math.fsum((a2 * etam)[col]),
        "kinetic_energy": 0.5 * math.fsum(np.concatenate([(vol_c * u * u)[wu], (vol_v * v * v)[wv]])),
        "max_abs_u": np.abs(u[wu]).max(), "max_abs_v": np.abs(v[wv]).max(),
        "max_abs_w": np.abs(wf[face_wet]).max(),
        "t_min": T[wet].min(), "t_max": T[wet].max(),
        "eta_min": eta[col].min(), "eta_max": eta[col].max(),
        "nonfinite": 0.0, "cfl_adv": cfl, "wet_area": math.fsum(a2[col]),
        "cfl_bt": np.max(np.where(col, np.sqrt(w.g * (wet * dz[:, None, None]).sum(axis=0)) * (w.dt / w.n_substeps)
                                  * np.sqrt(1.0 / dxc[:, None] ** 2 + 1.0 / dy ** 2), 0.0)),
    }


@pytest.mark.parametrize("case", ["latlon", "beta"])
def test_diagnostics_from_their_definitions(case):
    if case == "latlon":
        w = small_latlon(nx=30, ny=18, nz=7, tau0=0.3)
    else:
        w = inputs.BETA_BASIN_64.replace(nx=20, ny=14, nz=5, tau0=0.4)
    inp = inputs.make_inputs(w)
    kb, dz = inp["kbottom"], inp["dz"]
    m = oracle.OracleModel.from_inputs(w, inp)
    steps = 4
    m.step(steps)
    got = m.diagnostics()
    exp = _expected(w, m, kb, dz, steps)
    for name, e in exp.items():
        g = got[name]
        if name in ("tracer_content", "volume", "volume_mean", "kinetic_energy", "wet_area"):
            assert abs(g - e) <= 1e-14 * max(abs(e), 1e-300) + 1e-300, (name, g, e)
        elif name in ("max_abs_w", "cfl_adv", "cfl_bt"):
            assert abs(g - e) <= 1e-12 * abs(e), (name, g, e)  # w from a differently ordered sum
        else:
            assert g == e, (name, g, e)
    assert got["kinetic_energy"] > 0 and got["max_abs_w"] > 0


def test_nonfinite_counts_cells_and_columns():
    w = small_latlon(nx=12, ny=8, nz=4)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    m.step(1)
    assert m.diagnostics()["nonfinite"] == 0
    u, T, eta, U = m.get("u"), m.get("T"), m.get("eta"), m.get("U")
    u[2, 3, 4] = np.nan        # one cell through u
    T[2, 3, 4] = np.inf        # the same cell through T: still one cell
    T[1, 5, 6] = -np.inf       # a second cell
    eta[4, 4] = np.nan         # one column
    U[4, 4] = np.nan           # the same column
    for n, a in (("u", u), ("T", T), ("eta", eta), ("U", U)):
        m.set(n, a)
    assert m.diagnostics()["nonfinite"] == 3
