"""Pins of the oracle's tendency operators against closed forms and invariants:
Coriolis energy neutrality and uniform-flow values, the pressure gradient of a
linear temperature field, fifth-order convergence of the assembled tracer and
momentum advection, the vertical flux, consistency of the vertical transport
with the horizontal fluxes, and momentum conservation of the advection."""
import math

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, metrics, small_latlon


def _random_state(m, w, kb, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    shape = (w.nz, w.ny, w.nx)
    m.set("u", scale * rng.normal(size=shape))
    m.set("v", scale * rng.normal(size=shape))
    return m.get("u"), m.get("v")


def test_coriolis_energy_neutral_on_sphere_with_bathymetry():
    w = small_latlon()
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    u, v = _random_state(m, w, inp["kbottom"], 11)
    gu, gv, _ = m.tendencies(oracle.TERM_COR)
    dxc, dxv, dy, area = metrics(w)
    dz = inp["dz"]
    vu = area[None, :, None] * dz[:, None, None]
    vv = (dxv[:-1] * dy)[None, :, None] * dz[:, None, None]
    terms = np.concatenate([(vu * u * gu).ravel(), (vv * v * gv).ravel()])
    assert abs(terms.sum()) <= 1e-13 * np.abs(terms).sum()
    assert np.abs(terms).sum() > 0


def test_coriolis_uniform_flow_f_plane():
    w = inputs.Workload(name="fp", nx=6, ny=5, nz=3, periodic_x=True, periodic_y=True,
                        f0=1e-4, beta=0.0, tau0=0.0, noise_std=0.0)
    m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
    shape = (w.nz, w.ny, w.nx)
    m.set("u", np.full(shape, 0.2))
    m.set("v", np.full(shape, -0.05))
    gu, gv, _ = m.tendencies(oracle.TERM_COR)
    assert np.allclose(gu, 1e-4 * -0.05, rtol=1e-14, atol=0)
    assert np.allclose(gv, -1e-4 * 0.2, rtol=1e-14, atol=0)


@pytest.mark.parametrize("direction", ["x", "y"])
def test_pressure_gradient_of_linear_temperature(direction):
    """T = T0 + G x (or y): -dp/dx = g alpha G d_k at every wet interior face,
    d_k the depth of the layer centre."""
    w = inputs.Workload(name="pg", nx=8, ny=7, nz=5, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0)
    dz = inputs.layer_thickness(w)
    m = oracle.OracleModel(w, dz, inputs.wet_layers(w))
    G = 1e-6
    xc = (np.arange(w.nx) + 0.5) * w.dx
    yc = (np.arange(w.ny) + 0.5) * w.dy
    lin = xc[None, None, :] if direction == "x" else yc[None, :, None]
    T = 10.0 + G * lin + np.zeros((w.nz, w.ny, w.nx))
    m.set("T", T)
    gu, gv, _ = m.tendencies(oracle.TERM_PGF)
    depth = -inputs.layer_centre_z(w)
    expect = w.g * w.alpha * G * depth[:, None, None]
    if direction == "x":
        assert np.allclose(gu[:, :, 1:], np.broadcast_to(expect, gu[:, :, 1:].shape), rtol=1e-9, atol=0)
        assert np.all(gu[:, :, 0] == 0.0)
        assert np.max(np.abs(gv)) <= 1e-12 * np.max(np.abs(expect))
    else:
        assert np.allclose(gv[:, 1:, :], np.broadcast_to(expect, gv[:, 1:, :].shape), rtol=1e-9, atol=0)
        assert np.max(np.abs(gu)) <= 1e-12 * np.max(np.abs(expect))


def _order(errs):
    return [math.log2(errs[q] / errs[q + 1]) for q in range(len(errs) - 1)]


def _sine_avg(n, L):
    h = L / n
    x = (np.arange(n) + 0.5) * h
    k = 2 * math.pi / L
    avg = (np.cos(k * (x - h / 2)) - np.cos(k * (x + h / 2))) / (k * h)
    davg = (np.sin(k * (x + h / 2)) - np.sin(k * (x - h / 2))) / h  # average of d/dx sin
    return avg, davg


@pytest.mark.parametrize("direction", ["x", "y"])
def test_tracer_advection_fifth_order(direction):
    errs = []
    L = 1.0e6
    for n in (16, 32, 64, 128):
        nx, ny = (n, 2) if direction == "x" else (2, n)
        w = inputs.Workload(name="adv", nx=nx, ny=ny, nz=2, periodic_x=True, periodic_y=True,
                            dx=L / nx, dy=L / ny, depth=200.0, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0)
        m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
        avg, davg = _sine_avg(n, L)
        shape = (w.nz, w.ny, w.nx)
        if direction == "x":
            T = np.broadcast_to(avg[None, None, :], shape).copy()
            m.set("u", np.full(shape, 0.7))
            exact = -0.7 * np.broadcast_to(davg[None, None, :], shape)
        else:
            T = np.broadcast_to(avg[None, :, None], shape).copy()
            m.set("v", np.full(shape, -0.4))
            exact = 0.4 * np.broadcast_to(davg[None, :, None], shape)
        m.set("T", T)
        _, _, gt = m.tendencies(oracle.TERM_ADV)
        errs.append(np.mean(np.abs(gt - exact)))
    assert min(_order(errs)[1:]) >= 4.8, errs


@pytest.mark.parametrize("case", ["u_by_v", "v_by_u"])
def test_momentum_advection_fifth_order(case):
    """v0 uniform and u(y): ADV_u = -v0 du/dy. u0 uniform and v(x): ADV_v = -u0 dv/dx."""
    errs = []
    L = 1.0e6
    for n in (16, 32, 64, 128):
        nx, ny = (2, n) if case == "u_by_v" else (n, 2)
        w = inputs.Workload(name="madv", nx=nx, ny=ny, nz=2, periodic_x=True, periodic_y=True,
                            dx=L / nx, dy=L / ny, depth=200.0, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0)
        m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
        avg, davg = _sine_avg(n, L)
        shape = (w.nz, w.ny, w.nx)
        if case == "u_by_v":
            m.set("u", 0.05 * np.broadcast_to(avg[None, :, None], shape))
            m.set("v", np.full(shape, 0.6))
            gu, _, _ = m.tendencies(oracle.TERM_ADV)
            err = gu - (-0.6 * 0.05 * np.broadcast_to(davg[None, :, None], shape))
        else:
            # v lives on south faces at cell-centre x: averages over [x_{i-1/2}, x_{i+1/2}]
            m.set("v", 0.05 * np.broadcast_to(avg[None, None, :], shape))
            m.set("u", np.full(shape, -0.3))
            _, gv, _ = m.tendencies(oracle.TERM_ADV)
            err = gv - (0.3 * 0.05 * np.broadcast_to(davg[None, None, :], shape))
        errs.append(np.mean(np.abs(err)))
    assert min(_order(errs)[1:]) >= 4.8, errs


def test_vertical_flux_fifth_order():
    errs = []
    for n in (32, 64, 128, 256):
        avg, davg = _sine_avg(n, 1.0)
        wet = np.ones(n, dtype=np.int32)
        wf = np.full(n + 1, 0.8)
        wf[0] = wf[-1] = 0.0
        f = oracle.column_zflux(avg, wet, wf)
        div = -(f[1:] - f[:-1]) * n
        inner = slice(4, n - 4)
        errs.append(np.mean(np.abs(div[inner] + 0.8 * davg[inner])))
    assert min(_order(errs)[1:]) >= 4.8, errs


def test_uniform_tracer_preserved_below_surface():
    """With T uniform, the flux-form tendency vanishes in every wet layer below
    the top (the vertical transport is the one continuity gives); in the top
    layer it equals T0 W_top / V with W_top = -(column sum of horizontal
    transport divergence), because the surface face carries no advective flux."""
    w = small_latlon(restore_days=0.0)
    inp = inputs.make_inputs(w)
    T0 = 17.25
    inp["T0"] = np.full((w.nz, w.ny, w.nx), T0)
    m = oracle.OracleModel.from_inputs(w, inp)
    u, v = _random_state(m, w, inp["kbottom"], 5)
    _, _, gt = m.tendencies(oracle.TERM_ADV)
    wet, mu, mv = masks(w, inp["kbottom"])
    dxc, dxv, dy, area = metrics(w)
    dz = inp["dz"]
    U3 = u * mu * dy * dz[:, None, None]
    V3 = v * mv * dxv[None, :-1, None] * dz[:, None, None]
    V3n = np.concatenate([V3[:, 1:, :], np.zeros_like(V3[:, :1, :])], axis=1)  # bounded north edge
    div = (np.roll(U3, -1, axis=2) - U3) + (V3n - V3)
    vol = area[None, :, None] * dz[:, None, None]
    scale = T0 * np.max(np.abs(div)) / np.min(vol)
    below = wet.copy()
    below[-1] = False
    assert np.max(np.abs(gt[below])) <= 1e-12 * scale
    top = wet[-1]
    w_top = -div.sum(axis=0)
    expect = T0 * w_top / vol[-1]
    assert np.max(np.abs(gt[-1][top] - expect[top])) <= 1e-11 * scale
    assert np.max(np.abs(expect[top])) > 1e-6 * scale


def test_momentum_advection_conserves_momentum_periodic_flat():
    w = inputs.Workload(name="mc", nx=12, ny=10, nz=5, periodic_x=True, periodic_y=True,
                        f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0)
    m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
    rng = np.random.default_rng(2)
    shape = (w.nz, w.ny, w.nx)
    m.set("u", 0.5 * rng.normal(size=shape))
    m.set("v", 0.5 * rng.normal(size=shape))
    gu, gv, _ = m.tendencies(oracle.TERM_ADV)
    for g in (gu, gv):
        assert abs(g.sum()) <= 1e-13 * np.abs(g).sum()
        assert np.abs(g).sum() > 0


def test_wind_and_restoring_terms():
    w = small_latlon()
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    gu, gv, _ = m.tendencies(oracle.TERM_WIND)
    wet, mu, mv = masks(w, inp["kbottom"])
    dz = inp["dz"]
    expect = inp["taux"] / (w.rho0 * dz[-1])
    assert np.allclose(gu[-1][mu[-1]], expect[mu[-1]], rtol=1e-15)
    assert np.all(gu[:-1] == 0) and np.all(gu[-1][~mu[-1]] == 0) and np.all(gv == 0)
    _, _, gt = m.tendencies(oracle.TERM_RESTORE)
    tau = w.restore_days * 86400.0
    exp_t = (inp["tstar"] - inp["T0"][-1]) / tau
    assert np.allclose(gt[-1][wet[-1]], exp_t[wet[-1]], rtol=1e-14)
    assert np.all(gt[:-1] == 0)


def test_coriolis_metric_term_uniform_zonal_flow():
    """Uniform zonal flow u0 on the sphere: the meridional acceleration is
    -(f + u0 tan(phi)/a) u0 at the v-point latitude, to second order in dphi."""
    w = small_latlon(nx=72, ny=120, nz=2, bathymetry="flat", y0=-60.0, dy=1.0, depth=1000.0)
    m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
    u0 = 100.0
    m.set("u", np.full((w.nz, w.ny, w.nx), u0))
    _, gv, _ = m.tendencies(oracle.TERM_COR)
    lat_s = np.radians(w.y0 + np.arange(w.ny) * w.dy)
    expect = -(2 * w.omega * np.sin(lat_s) + u0 * np.tan(lat_s) / w.radius) * u0
    got = gv[0, 1:, 0]
    err = np.abs(got - expect[1:]) / np.max(np.abs(expect))
    assert np.max(err) < 1e-3
    without_metric = -(2 * w.omega * np.sin(lat_s)) * u0
    assert np.max(np.abs(without_metric[1:] - expect[1:])) / np.max(np.abs(expect)) > 1e-2


@pytest.mark.parametrize("case", ["uu_x", "vv_y", "uv_y", "vu_x"])
def test_nonlinear_momentum_flux_second_order(case):
    """One layer (no vertical flux), doubly periodic: the flux-form advection of
    a varying velocity converges to -d(u u)/dx, -d(v v)/dy, -d(v u)/dy or
    -d(u v)/dx at second order (the transports are averaged to the control
    volume faces, a second-order step)."""
    errs = []
    L = 2.0e6
    for n in (32, 64, 128, 256):
        along_x = case in ("uu_x", "vu_x")
        nx, ny = (n, 2) if along_x else (2, n)
        w = inputs.Workload(name="nl", nx=nx, ny=ny, nz=1, periodic_x=True, periodic_y=True,
                            dx=L / nx, dy=L / ny, depth=100.0, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0)
        m = oracle.OracleModel(w, inputs.layer_thickness(w), inputs.wet_layers(w))
        h = L / n
        k = 2 * math.pi / L
        xc = (np.arange(n) + 0.5) * h   # cell centres
        xf = np.arange(n) * h           # west / south faces
        A, B = 0.8, 0.3

        def prof(x):
            return 1.0 + A * np.sin(k * x) + B * np.cos(2 * k * x)

        def avg(x0):  # average of prof over [x0 - h/2, x0 + h/2]
            F = lambda x: x - A * np.cos(k * x) / k + B * np.sin(2 * k * x) / (2 * k)
            return (F(x0 + h / 2) - F(x0 - h / 2)) / h

        shape = (1, ny, nx)
        if case == "uu_x":    # u on faces x_{i-1/2}, CV between centres i-1 and i
            m.set("u", avg(xf).reshape(1, 1, n) * np.ones(shape))
            gu, _, _ = m.tendencies(oracle.TERM_ADV)
            exact = -(prof(xf + h / 2) ** 2 - prof(xf - h / 2) ** 2) / h
            got = gu[0, 0, :]
        elif case == "vv_y":
            m.set("v", avg(xf).reshape(1, n, 1) * np.ones(shape))
            _, gv, _ = m.tendencies(oracle.TERM_ADV)
            exact = -(prof(xf + h / 2) ** 2 - prof(xf - h / 2) ** 2) / h
            got = gv[0, :, 0]
        elif case == "uv_y":  # u(y), v(y): d(v u)/dy, u CV spans faces y_{j-1/2}..y_{j+1/2}
            m.set("u", avg(xc).reshape(1, n, 1) * np.ones(shape))
            m.set("v", 0.5 * prof(xf).reshape(1, n, 1) * np.ones(shape))
            gu, _, _ = m.tendencies(oracle.TERM_ADV)
            exact = -(0.5 * prof(xf + h) * prof(xf + h) - 0.5 * prof(xf) * prof(xf)) / h
            got = gu[0, :, 0]
        else:                 # v(x), u(x): d(u v)/dx, v CV spans faces x_{i-1/2}..x_{i+1/2}
            m.set("v", avg(xc).reshape(1, 1, n) * np.ones(shape))
            m.set("u", 0.5 * prof(xf).reshape(1, 1, n) * np.ones(shape))
            _, gv, _ = m.tendencies(oracle.TERM_ADV)
            exact = -(0.5 * prof(xf + h) * prof(xf + h) - 0.5 * prof(xf) * prof(xf)) / h
            got = gv[0, 0, :]
        errs.append(np.mean(np.abs(got - exact)))
    orders = _order(errs)
    assert min(orders[1:]) >= 1.9, (orders, errs)
