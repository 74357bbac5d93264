"""Pins of salinity and the nonlinear equation of state in the oracle.

Reading: the paper's realistic runs carry heat and salt (Sec. 6) and name no
equation of state; S is a second tracer advected, restored and diffused like
T, and the buoyancy follows the simplified seawater equation of state of
Roquet et al. (2015):
rho' = -a0 (1 + lambda1 Ta/2 + mu1 z) Ta + b0 (1 - lambda2 Sa/2 - mu2 z) Sa - nu Ta Sa,
b = -g rho'/rho0, with Ta = T - 10, Sa = S - 35 and z the depth.

- worked values of b at three (T, S, z) points (the arithmetic is spelt out);
- properties the form fixes: the reference water is neutral, warmer water is
  lighter and more so at depth (thermobaricity), and mixing two water masses
  of equal density gives denser water (cabbeling);
- with the nonlinear, salt and pressure terms off it reduces to the linear
  temperature equation of state: a step equals the temperature-only model's;
- the pressure gradient of a salinity linear in x or y is g b0 G d / rho0 at
  every layer centre of depth d (linear equation of state in S);
- salt content is conserved to round-off; a horizontally uniform T, S
  stratification stays at rest;
- with nothing but S in the buoyancy, S drives the same flow T does when the
  equations of state map one onto the other.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, metrics, small_latlon

EOS = inputs.Workload.__dataclass_fields__["eos"].default


def _salty(**kw):
    base = dict(salinity=True)
    base.update(kw)
    return small_latlon(**base)


def test_equation_of_state_worked_values():
    w = _salty(nx=4, ny=3, nz=2)
    m = oracle.OracleModel.from_inputs(w, inputs.make_inputs(w))
    g, r0 = w.g, w.rho0
    # T = 20, S = 35, z = 0: Ta = 10, rho' = -0.1655 (1 + 0.02976 * 10) * 10 = -2.147528
    assert m.buoyancy(20.0, 35.0, 0.0) == pytest.approx(-g * -2.147528 / r0, rel=1e-14)
    # T = 10, S = 36, z = 0: Sa = 1, rho' = 0.76554 (1 - 0.00027457) = 0.765329805682
    assert m.buoyancy(10.0, 36.0, 0.0) == pytest.approx(-g * 0.765329805682 / r0, rel=1e-12)
    # T = 2, S = 34.5, z = 1000: Ta = -8, Sa = -0.5
    #   -0.1655 (1 - 0.23808 + 0.1497)(-8) = 1.20698488
    #   0.76554 (1 + 0.000137285 - 0.01109)(-0.5) = -0.378577629279
    #   -0.0024341 (-8)(-0.5) = -0.0097364          rho' = 0.818670850721
    assert m.buoyancy(2.0, 34.5, 1000.0) == pytest.approx(-g * 0.818670850721 / r0, rel=1e-12)
    assert m.buoyancy(10.0, 35.0, 0.0) == 0.0


def test_equation_of_state_properties():
    w = _salty(nx=4, ny=3, nz=2)
    m = oracle.OracleModel.from_inputs(w, inputs.make_inputs(w))
    b = m.buoyancy
    # warmer is lighter, saltier is denser
    assert b(12.0, 35.0, 0.0) > b(11.0, 35.0, 0.0) and b(10.0, 35.5, 0.0) < b(10.0, 35.0, 0.0)
    # thermobaricity: the thermal expansion grows with depth
    assert (b(11.0, 35.0, 3000.0) - b(10.0, 35.0, 3000.0)) > (b(11.0, 35.0, 0.0) - b(10.0, 35.0, 0.0))
    # cabbeling: two waters of equal density, mixed half and half, give denser water
    t1, s1, t2 = 2.0, 34.0, 18.0
    # salinity of the warm water that matches the cold water's buoyancy (bisection on S)
    lo, hi = 30.0, 40.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if b(t2, mid, 0.0) > b(t1, s1, 0.0):
            lo = mid
        else:
            hi = mid
    s2 = 0.5 * (lo + hi)
    assert abs(b(t2, s2, 0.0) - b(t1, s1, 0.0)) < 1e-15
    assert b(0.5 * (t1 + t2), 0.5 * (s1 + s2), 0.0) < b(t1, s1, 0.0) - 1e-6


def test_reduces_to_the_linear_temperature_equation_of_state():
    """a0 = alpha rho0, every other coefficient 0, t0 = t_ref: S is passive
    and the step is the temperature-only step to rounding."""
    base = small_latlon(nx=24, ny=14, nz=6, tau0=0.2)
    a0 = base.alpha * base.rho0
    lin = base.replace(salinity=True, eos=(a0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, base.t_ref, 35.0))
    inp_t = inputs.make_inputs(base)
    inp_s = inputs.make_inputs(lin)
    assert np.array_equal(inp_t["T0"], inp_s["T0"])
    mt = oracle.OracleModel.from_inputs(base, inp_t)
    ms = oracle.OracleModel.from_inputs(lin, inp_s)
    mt.step(4)
    ms.step(4)
    wet, mu, mv = masks(base, inp_t["kbottom"])
    for name, mask in (("u", mu), ("v", mv), ("T", wet)):
        a, e = ms.get(name)[mask], mt.get(name)[mask]
        assert np.linalg.norm(a - e) <= 1e-12 * np.linalg.norm(e), name
    for name in ("eta", "U", "V"):
        a, e = ms.get(name), mt.get(name)
        assert np.linalg.norm(a - e) <= 1e-11 * np.linalg.norm(e), name


@pytest.mark.parametrize("direction", ["x", "y"])
def test_pressure_gradient_of_linear_salinity(direction):
    """S = 35 + G x (or y), T = 10, linear equation of state in S: -dp/dx =
    g b0 G d / rho0 (saltier water is denser, so the flow is pushed towards
    lower salinity: -dp/dx = -db/dx d with db/dx = -g b0 G / rho0)."""
    b0 = 0.8
    w = inputs.Workload(name="pgs", nx=8, ny=7, nz=5, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0,
                        salinity=True, eos=(0.0, b0, 0.0, 0.0, 0.0, 0.0, 0.0, 10.0, 35.0))
    dz = inputs.layer_thickness(w)
    m = oracle.OracleModel(w, dz, inputs.wet_layers(w))
    G = 1e-6
    xc = (np.arange(w.nx) + 0.5) * w.dx
    yc = (np.arange(w.ny) + 0.5) * w.dy
    lin = xc[None, None, :] if direction == "x" else yc[None, :, None]
    m.set("T", np.full((w.nz, w.ny, w.nx), 10.0))
    m.set("S", 35.0 + G * lin + np.zeros((w.nz, w.ny, w.nx)))
    gu, gv, _ = m.tendencies(oracle.TERM_PGF)
    depth = -inputs.layer_centre_z(w)
    expect = -w.g * b0 * G / w.rho0 * depth[:, None, None]
    if direction == "x":
        assert np.allclose(gu[:, :, 1:], np.broadcast_to(expect, gu[:, :, 1:].shape), rtol=1e-9, atol=0)
        assert np.max(np.abs(gv)) <= 1e-12 * np.max(np.abs(expect))
    else:
        assert np.allclose(gv[:, 1:, :], np.broadcast_to(expect, gv[:, 1:, :].shape), rtol=1e-9, atol=0)
        assert np.max(np.abs(gu)) <= 1e-12 * np.max(np.abs(expect))


def test_salt_content_conserved_and_tendency_of_uniform_salt():
    w = _salty(nx=30, ny=16, nz=6, tau0=0.3, restore_days=0.0)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    wet, _, _ = masks(w, inp["kbottom"])
    _, _, _, area = metrics(w)
    vol = area[None, :, None] * inp["dz"][:, None, None] * np.ones((1, 1, w.nx))
    s0 = math.fsum((vol * m.get("S"))[wet])
    assert m.diagnostics()["salt_content"] == pytest.approx(s0, rel=1e-15)
    m.step(8)
    s1 = math.fsum((vol * m.get("S"))[wet])
    assert abs(s1 - s0) <= 1e-13 * abs(s0)
    assert m.diagnostics()["salt_content"] == pytest.approx(s1, rel=1e-14)
    assert m.diagnostics()["max_abs_u"] > 0  # the flow did move


def test_stratified_rest_state_stays_at_rest():
    w = inputs.BETA_BASIN_64.replace(nx=12, ny=10, nz=8, tau0=0.0, noise_std=0.0, noise_std_s=0.0, salinity=True)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    m.step(10)
    for name in ("u", "v", "U", "V"):
        assert np.all(m.get(name) == 0.0), name
    S = m.get("S")
    assert np.all(S == S[:, :1, :1])
    assert not np.array_equal(S, inp["S0"])  # vertical diffusion acted on S


def test_salinity_drives_what_temperature_drives():
    """Salt standing in for heat: a model whose buoyancy comes from T alone
    (a0 = alpha rho0) and one whose buoyancy comes from S alone (b0 = -a0,
    reference salinity 10) with S holding the first model's T field give the
    same flow, bitwise, and S follows T. (An offset S = T + c would not: under
    the linear free surface a uniform tracer is not preserved in the top layer.)"""
    base = small_latlon(nx=20, ny=12, nz=5, tau0=0.2, restore_days=0.0)
    a0 = base.alpha * base.rho0
    tw = base.replace(salinity=True, eos=(a0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 10.0, 35.0))
    sw = base.replace(salinity=True, eos=(0.0, -a0, 0.0, 0.0, 0.0, 0.0, 0.0, 10.0, 10.0))
    inp = inputs.make_inputs(tw)
    mt = oracle.OracleModel.from_inputs(tw, inp)
    mt.set("S", np.full_like(inp["T0"], 35.0))
    inp_s = dict(inp)
    inp_s["S0"] = inp["T0"].copy()
    inp_s["T0"] = np.full_like(inp["T0"], 10.0)
    ms = oracle.OracleModel.from_inputs(sw, inp_s)
    mt.step(3)
    ms.step(3)
    for name in ("u", "v", "eta", "U", "V"):
        assert np.array_equal(ms.get(name), mt.get(name)), name
    assert np.array_equal(ms.get("S"), mt.get("T"))
