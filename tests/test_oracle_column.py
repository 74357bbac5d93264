"""Pins of the oracle's column operators: tridiagonal solve, implicit vertical
diffusion (backward Euler, paper Sec. 5.2) and the hydrostatic pressure
diagnostic (paper Sec. 5.1)."""
import math

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16])
def test_thomas_matches_dense_solve(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        a = rng.uniform(-1, 0, size=n)
        c = rng.uniform(-1, 0, size=n)
        a[0] = 0.0
        c[-1] = 0.0
        b = np.abs(a) + np.abs(c) + rng.uniform(0.1, 2.0, size=n)
        d = rng.normal(size=n)
        A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        x = oracle.thomas(a, b, c, d)
        ref = np.linalg.solve(A, d)
        assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def _column_workload(nz, kappa, dt=1200.0):
    return inputs.Workload(name="col", nx=2, ny=2, nz=nz, periodic_x=True, periodic_y=True,
                           dx=50e3, dy=50e3, depth=nz * 100.0, f0=0.0, beta=0.0, kappa=kappa,
                           dt=dt, n_substeps=10, tau0=0.0, noise_std=0.0)


@pytest.mark.parametrize("mode", [1, 2, 5])
def test_diffusion_eigenmode_decay(mode):
    """One backward-Euler solve multiplies a Neumann cosine mode by
    1 / (1 + dt kappa (4/dz^2) sin^2(pi m / (2 nz)))."""
    nz, kappa, dt = 16, 1e-2, 1200.0
    w = _column_workload(nz, kappa, dt)
    dz = np.full(nz, 100.0)
    m = oracle.OracleModel(w, dz, np.full((2, 2), nz, dtype=np.int32))
    k = np.arange(nz)
    prof = np.cos(math.pi * mode * (k + 0.5) / nz)
    T = np.broadcast_to(prof[:, None, None], (nz, 2, 2)).copy()
    u = 0.1 * T
    m.set("T", T)
    m.set("u", u)
    m.set("v", -0.2 * T)
    m.step(1)
    fac = 1.0 / (1.0 + dt * kappa * 4.0 / 100.0 ** 2 * math.sin(math.pi * mode / (2 * nz)) ** 2)
    for name, ref in (("T", T), ("u", u), ("v", -0.2 * T)):
        got = m.get(name)
        assert np.max(np.abs(got - fac * ref)) <= 1e-13 * np.max(np.abs(ref)), name


def test_diffusion_preserves_column_integral():
    nz = 12
    w = _column_workload(nz, 5e-2)
    dz = np.linspace(50, 300, nz)
    m = oracle.OracleModel(w.replace(depth=float(dz.sum())), dz, np.full((2, 2), nz, dtype=np.int32))
    rng = np.random.default_rng(0)
    prof = rng.normal(size=nz)
    T = np.broadcast_to(prof[:, None, None], (nz, 2, 2)).copy()
    m.set("T", T)
    m.step(1)
    got = m.get("T")[:, 0, 0]
    assert abs(np.dot(dz, got) - np.dot(dz, prof)) <= 1e-14 * np.dot(dz, np.abs(prof))
    # and it is a genuine smoothing: the variance drops
    assert np.var(got) < np.var(prof)


def test_pressure_linear_profile():
    """dp/dz = b with p(0) = 0: trapezoids between centres are exact for linear b;
    the top half-layer uses the top-layer buoyancy."""
    nz = 10
    w = _column_workload(nz, 0.0)
    dz = np.linspace(80, 200, nz)
    m = oracle.OracleModel(w.replace(depth=float(dz.sum())), dz, np.full((2, 2), nz, dtype=np.int32))
    zc = np.cumsum(dz) - dz.sum() - 0.5 * dz
    T = 4.0 + 0.01 * zc
    m.set("T", np.broadcast_to(T[:, None, None], (nz, 2, 2)).copy())
    p = m.get("p")[:, 0, 0]
    ga = w.g * w.alpha
    b = ga * (T - w.t_ref)
    assert p[-1] == pytest.approx(-0.5 * dz[-1] * b[-1], rel=1e-15)
    # p_{k+1} - p_k = integral of b between the centres (exact for linear b)
    exact_diff = ga * (4.0 * (zc[1:] - zc[:-1]) + 0.005 * (zc[1:] ** 2 - zc[:-1] ** 2))
    assert np.allclose(p[1:] - p[:-1], exact_diff, rtol=1e-12, atol=0)


def test_pressure_second_order_convergence():
    """T = 20 exp(z/1000): the pressure error at fixed depth falls about 4x per halving of dz."""
    errs = []
    H = 4000.0
    for nz in (10, 20, 40, 80):
        w = _column_workload(nz, 0.0)
        dz = np.full(nz, H / nz)
        m = oracle.OracleModel(w.replace(depth=H), dz, np.full((2, 2), nz, dtype=np.int32))
        zc = np.cumsum(dz) - H - 0.5 * dz
        m.set("T", np.broadcast_to((20.0 * np.exp(zc / 1000.0))[:, None, None], (nz, 2, 2)).copy())
        p = m.get("p")[:, 0, 0]
        ga = w.g * w.alpha
        exact = -ga * 20.0 * 1000.0 * (1.0 - np.exp(zc / 1000.0))
        # compare at z = -2000 - dz/2 ... use interpolation to the centres at fixed depths
        errs.append(np.max(np.abs(p - exact)))
    ratios = [errs[q] / errs[q + 1] for q in range(3)]
    assert all(3.5 < r < 4.3 for r in ratios) and abs(ratios[-1] - 4.0) < 0.1, ratios


def test_diffusion_modes_follow_each_velocity_column_depth():
    """With uneven bathymetry every u (v) column is a Neumann problem over its own
    wet depth, min of the two neighbouring tracer columns across x (y). A
    first cosine mode over those levels decays by the closed-form factor.
    Velocities are tiny so advection (quadratic in them) stays below round-off."""
    nz, kappa, dt, dzv = 8, 2e-2, 1200.0, 100.0
    w = inputs.Workload(name="steps", nx=6, ny=5, nz=nz, periodic_x=True, periodic_y=True,
                        dx=50e3, dy=50e3, depth=nz * dzv, f0=0.0, beta=0.0, kappa=kappa, dt=dt,
                        n_substeps=10, tau0=0.0, noise_std=0.0, strat_t0=0.0)
    rng = np.random.default_rng(4)
    kb = rng.integers(2, nz + 1, size=(w.ny, w.nx)).astype(np.int32)
    m = oracle.OracleModel(w, np.full(nz, dzv), kb)
    amp = 1e-12
    fields = {}
    for name, kcol in (("u", np.minimum(kb, np.roll(kb, 1, axis=1))),
                       ("v", np.minimum(kb, np.roll(kb, 1, axis=0)))):
        f = np.zeros((nz, w.ny, w.nx))
        fac = np.zeros((w.ny, w.nx))
        for j in range(w.ny):
            for i in range(w.nx):
                K = kcol[j, i]
                q = np.arange(K)
                f[nz - K:, j, i] = amp * np.cos(np.pi * (q + 0.5) / K)
                fac[j, i] = 1.0 / (1.0 + dt * kappa * 4.0 / dzv ** 2 * np.sin(np.pi / (2 * K)) ** 2)
        fields[name] = (f, fac)
        m.set(name, f)
    m.step(1)
    for name, (f, fac) in fields.items():
        got = m.get(name)
        assert np.max(np.abs(got - fac[None] * f)) <= 1e-11 * amp, name
