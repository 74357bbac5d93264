"""Pins of the time stepping of the oracle's baroclinic step (paper Sec. 5.2:
implicit-explicit second-order Adams-Bashforth).

Reading. The tracer and every momentum term except the hydrostatic pressure
gradient take AB2 with offset chi; the pressure gradient is not extrapolated
but taken from the hydrostatic pressure of T^n + eps dt Ghat_T, the tracer
just predicted, weighted by eps (a forward-backward treatment of the internal
gravity waves). The pins:

- the scheme's characteristic roots for the oscillation pair that internal
  waves reduce to (h' = -i w u, u' = -i w h) stay inside the unit circle up to
  w dt ~ 1.3 with eps = 3/4 and chi = 0.1, while AB2 of both terms grows by
  ~1.5 per step at the w dt ~ 0.95 that the 1/12-degree grid reaches at 75S;
- one oracle step is exactly that composition: T^{n+1} = T^n + dt Ghat_T
  without diffusion, and the baroclinic part of u^{n+1}, v^{n+1} equals AB2 of
  the other tendencies plus the pressure gradient of T^n + eps dt Ghat_T, each
  tendency taken from the oracle's stage entry point on the given state;
- windows of the benchmarked grids where internal waves are fastest relative
  to the grid (75S at 1/12 degree, 80S at 1/4 degree) and an equatorial window
  stay finite and bounded for 200 steps.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, small_latlon


def _roots(theta, chi, eps, extrapolate_pgf=False):
    """Moduli of the characteristic roots of one step for h' = -i w u, u' = -i w h.

    State (h^n, u^n, h^{n-1}, u^{n-1}); h takes AB2. u takes either AB2 too
    (extrapolate_pgf) or the pressure of h^n + eps (h^{n+1} - h^n)."""
    a, b, t = 1.5 + chi, 0.5 + chi, theta
    row_h = np.array([1.0, -1j * t * a, 0.0, 1j * t * b])
    if extrapolate_pgf:
        row_u = np.array([-1j * t * a, 1.0, 1j * t * b, 0.0])
    else:
        tfb = eps * row_h + (1.0 - eps) * np.array([1.0, 0.0, 0.0, 0.0])
        row_u = np.array([0.0, 1.0, 0.0, 0.0], dtype=complex) - 1j * t * tfb
    M = np.array([row_h, row_u, [1, 0, 0, 0], [0, 1, 0, 0]], dtype=complex)
    return np.abs(np.linalg.eigvals(M))


def test_forward_backward_pressure_keeps_internal_waves_bounded():
    thetas = np.linspace(0.01, 1.3, 130)
    worst = max(_roots(t, 0.1, 0.75).max() for t in thetas)
    assert worst <= 1.0 + 1e-12, worst
    # AB2 of the pressure gradient as well: the growth seen at 75S (about 1.5 per step)
    grow = _roots(0.95, 0.1, 0.0, extrapolate_pgf=True).max()
    assert 1.4 < grow < 1.7, grow
    # long waves are barely damped: a few 1e-4 per step at w dt = 0.05
    assert 1.0 - _roots(0.05, 0.1, 0.75).max() < 1e-3


def _depth_mean_removed(a, wet, dz):
    """a minus its dz-weighted mean over the wet levels of each column."""
    h = (wet * dz[:, None, None]).sum(axis=0)
    s = (a * wet * dz[:, None, None]).sum(axis=0)
    mean = np.where(h > 0, s / np.where(h > 0, h, 1.0), 0.0)
    return np.where(wet, a - mean[None], 0.0)


@pytest.mark.parametrize("eps", [0.0, 0.75, 1.0])
def test_step_is_ab2_plus_forward_backward_pressure(eps):
    w = small_latlon(nx=24, ny=16, nz=8, kappa=0.0, pgf_weight=eps, dt=3600.0)
    inp = inputs.make_inputs(w)
    kb, dz = inp["kbottom"], inp["dz"]
    wet, wu, wv = masks(w, kb)
    rng = np.random.default_rng(7)
    shape = (w.nz, w.ny, w.nx)
    u0 = np.where(wu, 0.05 * rng.standard_normal(shape), 0.0)
    v0 = np.where(wv, 0.05 * rng.standard_normal(shape), 0.0)
    T0 = inp["T0"] + 0.3 * rng.standard_normal(shape)
    hist = {n: 1e-6 * rng.standard_normal(shape) for n in ("gu_prev", "gv_prev", "gt_prev")}

    def model(T):
        m = oracle.OracleModel.from_inputs(w, inp)
        m.set("u", u0)
        m.set("v", v0)
        m.set("T", T)
        for n, a in hist.items():
            m.set(n, a)
        m.first_step = False
        return m

    chi, dt = w.chi, w.dt
    ab2 = lambda g, prev: (1.5 + chi) * g - (0.5 + chi) * prev
    # tendencies of the state at step n, from the stage entry point
    gu, gv, gt = model(T0).tendencies(oracle.TERM_ALL & ~oracle.TERM_PGF)
    gt_hat = ab2(gt, hist["gt_prev"])
    t_fb = T0 + eps * dt * gt_hat
    pu, pv, _ = model(t_fb).tendencies(oracle.TERM_PGF)
    u_star = u0 + dt * (ab2(gu, hist["gu_prev"]) + pu)
    v_star = v0 + dt * (ab2(gv, hist["gv_prev"]) + pv)

    m = model(T0)
    m.step(1)
    T1 = m.get("T")
    scale = np.abs(T0[wet]).max()
    assert np.abs(T1 - (T0 + dt * gt_hat))[wet].max() <= 1e-13 * scale
    for got, exp, mask in ((m.get("u"), u_star, wu), (m.get("v"), v_star, wv)):
        d = _depth_mean_removed(got, mask, dz) - _depth_mean_removed(exp, mask, dz)
        assert np.abs(d).max() <= 1e-12 * np.abs(exp[mask]).max()
    # the AB2 histories are the new tendencies, the pressure gradient not among them
    for name, g in (("gu_prev", gu), ("gv_prev", gv), ("gt_prev", gt)):
        assert np.array_equal(m.get(name), g), name


def _bounded_window(args):
    name, nx, ny, lon0, lat0, steps = args
    base = inputs.WORKLOADS[name]
    w = base.replace(name=f"{name}_window", nx=nx, ny=ny, periodic_x=False, x0=lon0, y0=lat0)
    m = oracle.OracleModel.from_inputs(w, inputs.make_inputs(w))
    m.step(steps)
    d = m.diagnostics()
    m.close()
    return d


@pytest.mark.slow
def test_high_latitude_windows_stay_bounded():
    """200 steps of the benchmarked grids where their meridians converge most, and at the equator."""
    jobs = [("latlon_4320x1800x100", 64, 32, 150.0, -75.0, 200),
            ("latlon_4320x1800x100", 64, 32, 150.0, -10.0, 200),
            ("latlon_1440x600x50", 64, 32, 150.0, -80.0, 200)]
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        results = list(ex.map(_bounded_window, jobs))
    for job, d in zip(jobs, results):
        assert d["nonfinite"] == 0, job
        assert d["max_abs_u"] < 1.0 and d["max_abs_v"] < 1.0, (job, d["max_abs_u"], d["max_abs_v"])
        assert max(abs(d["eta_min"]), abs(d["eta_max"])) < 1.0, job
        assert d["cfl_adv"] < 0.2, job


def test_stages_in_turn_equal_a_step():
    """The four stages run one by one give bitwise what a step gives."""
    w = small_latlon(nx=20, ny=12, nz=6)
    inp = inputs.make_inputs(w)
    a = oracle.OracleModel.from_inputs(w, inp)
    b = oracle.OracleModel.from_inputs(w, inp)
    a.set_convective(0.5)
    b.set_convective(0.5)
    for n in range(3):
        a.step(1)
        for st in (oracle.STAGE_MIXING, oracle.STAGE_TENDENCY, oracle.STAGE_BAROTROPIC, oracle.STAGE_COLUMN):
            b.run_stage(st)
        b.first_step = False
        for name in ("u", "v", "T", "eta", "U", "V", "U_mean", "gu_prev", "gt_prev"):
            assert np.array_equal(a.get(name), b.get(name)), (n, name)
