"""Physics pins of the oracle's full step: what the equations fix independently
of the discretisation details (paper Sec. 5.2, 5.3).

- a resting stratified ocean stays at rest; every column then only diffuses;
- tracer content and free-surface volume are conserved to round-off (flux form);
- the free surface moves by the divergence of the averaged transport, and the
  3D velocity integrates to the barotropic transport after the correction;
- a basin-mode gravity wave has the discrete forward-backward frequency, close
  to the continuous sqrt(gH) value;
- a uniform inertial oscillation follows the split AB2 recurrence of the 3D flow and
  the barotropic mode (the depth mean taken from the substep-averaged transport);
- restarting from a saved state is bitwise identical to running straight on.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, metrics, small_latlon


def _window(ns):
    """Substep weights a_q (q = 1..M, M = Ns + Ns/2): cos^2(pi t), t = q/Ns - 1, |t| < 1/2, normalised."""
    M = ns + ns // 2
    q = np.arange(1, M + 1)
    t = q / ns - 1.0
    a = np.where(np.abs(t) < 0.5, np.cos(np.pi * t) ** 2, 0.0)
    return q, a / a.sum()


def test_substep_window():
    """The window is centred on t^{n+1}: weights sum to one, first moment Ns."""
    for ns in (1, 5, 30, 60):
        q, a = _window(ns)
        assert abs(a.sum() - 1.0) < 1e-15 and abs((q * a).sum() - ns) < 1e-12 * ns


def test_rest_state_stays_at_rest():
    w = inputs.BETA_BASIN_64.replace(nx=16, ny=12, noise_std=0.0, tau0=0.0)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    # a uniform surface offset exerts no force and is its own substep average
    m.set("eta", np.full((w.ny, w.nx), 0.125))
    m.step(20)
    for name in ("u", "v", "U", "V", "U_mean", "V_mean"):
        assert np.all(m.get(name) == 0.0), name
    # the weighted substep average of a constant surface is that constant to round-off
    for name in ("eta", "eta_mean"):
        assert np.max(np.abs(m.get(name) - 0.125)) <= 4e-16, name
    assert np.all(m.get("w") == 0.0)
    T = m.get("T")
    assert np.all(T == T[:, :1, :1])
    # a single column run the same way matches every column bitwise
    c = w.replace(nx=1, ny=1, periodic_x=True, periodic_y=True)
    mc = oracle.OracleModel.from_inputs(c, inputs.make_inputs(c))
    mc.step(20)
    assert np.array_equal(mc.get("T")[:, 0, 0], T[:, 0, 0])
    assert not np.array_equal(T[:, 0, 0], inp["T0"][:, 0, 0])  # diffusion acted


def _tracer_content(T, w, kb, dz):
    wet, _, _ = masks(w, kb)
    _, _, _, area = metrics(w)
    vol = area[None, :, None] * dz[:, None, None]
    return math.fsum((vol * T)[wet].ravel())


@pytest.mark.parametrize("case", ["beta", "latlon"])
def test_conservation_and_consistency(case):
    if case == "beta":
        w = inputs.BETA_BASIN_64.replace(nx=24, ny=20)
        nsteps = 12
    else:
        w = small_latlon(restore_days=0.0, tau0=0.2)
        nsteps = 6
    inp = inputs.make_inputs(w)
    kb, dz = inp["kbottom"], inp["dz"]
    m = oracle.OracleModel.from_inputs(w, inp)
    wet, mu, mv = masks(w, kb)
    dxc, dxv, dy, area = metrics(w)
    c0 = _tracer_content(inp["T0"], w, kb, dz)
    col = kb > 0
    for _ in range(nsteps):
        eta0 = m.get("eta")
        m.step(1)
        eta, U, V, u, v = (m.get(n) for n in ("eta", "U", "V", "u", "v"))
        Um, Vm, em = m.get("U_mean"), m.get("V_mean"), m.get("eta_mean")
        # volume: sum A eta and sum A eta_mean vanish to round-off
        for e in (eta, em):
            a = (area[:, None] * e)[col]
            assert abs(math.fsum(a)) <= 1e-12 * np.abs(a).sum() + 1e-300
        # eta^{n+1} - eta^n = -dt div(U_mean)
        Vn = np.concatenate([Vm[1:], np.zeros_like(Vm[:1])], axis=0) if not w.periodic_y else np.roll(Vm, -1, 0)
        Ue = np.roll(Um, -1, axis=1) if w.periodic_x else np.concatenate([Um[:, 1:], np.zeros_like(Um[:, :1])], 1)
        div = (dy * (Ue - Um) + dxv[1:, None] * Vn - dxv[:-1, None] * Vm) / area[:, None]
        resid = eta - eta0 + w.dt * div
        assert np.max(np.abs(resid)) <= 1e-12 * max(np.max(np.abs(eta)), 1e-30)
        # sum_k dz u = Ubar (the substep-averaged transport) after the correction
        for f, mk, B in ((u, mu, Um), (v, mv, Vm)):
            s = (dz[:, None, None] * f * mk).sum(axis=0)
            assert np.max(np.abs(s - B)) <= 1e-12 * max(np.max(np.abs(B)), 1e-30)
    c1 = _tracer_content(m.get("T"), w, kb, dz)
    assert abs(c1 - c0) <= 1e-12 * abs(c0)
    assert m.diagnostics()["nonfinite"] == 0
    assert np.max(np.abs(m.get("u"))) > 0


def test_gravity_wave_frequency_and_filter_damping():
    """Closed channel, flat 4 km, f = 0, T = 0: eta = 0.01 cos(pi x / L) is a
    discrete eigenmode. Each forward-backward substep rotates it by
    theta = 2 asin((c dtau/dx) sin(pi dx/(2L))), c = sqrt(gH); the step returns the
    window average sum_q a_q B^q, whose eigenvalues are R e^(+-i Ns theta) with
    R = sum_q a_q cos((q - Ns) theta) for weights symmetric about Ns. Sampled once
    per step, eta obeys eta^{n+1} = 2 R cos(Ns theta) eta^n - R^2 eta^{n-1}."""
    w = inputs.BETA_BASIN_64.replace(ny=2, nz=2, f0=0.0, beta=0.0, tau0=0.0, noise_std=0.0,
                                     strat_t0=0.0, kappa=0.0)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    L = w.nx * w.dx
    x = (np.arange(w.nx) + 0.5) * w.dx
    m.set("eta", np.broadcast_to(0.01 * np.cos(math.pi * x / L), (w.ny, w.nx)).copy())
    hist = [m.get("eta")]
    for _ in range(60):
        m.step(1)
        hist.append(m.get("eta"))
    e = np.array(hist).reshape(len(hist), -1)
    # least-squares fit of eta^{n+1} = A eta^n + B eta^{n-1} over all points and steps
    X = np.stack([e[1:-1].ravel(), e[:-2].ravel()], axis=1)
    (A, B), *_ = np.linalg.lstsq(X, e[2:].ravel(), rcond=None)
    R_obs = math.sqrt(-B)
    omega = math.acos(A / (2 * R_obs)) / w.dt
    c = math.sqrt(w.g * w.depth)
    ns = w.n_substeps
    dtau = w.dt / ns
    theta = 2.0 * math.asin(c * dtau / w.dx * math.sin(math.pi * w.dx / (2 * L)))
    q, a = _window(ns)
    R = float(np.sum(a * np.cos((q - ns) * theta)))
    assert abs(omega - ns * theta / w.dt) <= 1e-6 * omega
    assert abs(R_obs - R) <= 1e-9
    assert R < 1.0
    # and the continuous long-wave period 2L/c is within the discretisation error
    assert abs(2 * math.pi / omega - 2 * L / c) / (2 * L / c) < 2e-4


@pytest.mark.parametrize("chi", [0.0, 0.1])
def test_inertial_oscillation_follows_split_ab2(chi):
    """Uniform flow on a doubly periodic f-plane, q = u + i v of the 3D flow and
    Q = (U + i V) / H of the barotropic mode. With no surface slope the
    substeps add the slow forcing linearly, so with a = -i f dt and
    G = a [(3/2+chi) q^n - (1/2+chi) q^{n-1}] (a q^0 on the first step):
    Q^{n+1} = Q^n + G (the window is centred on t^{n+1}) and, the depth mean
    being replaced by the step's transport, q^{n+1} = Q^n + c G."""
    f, dt = 1e-4, 1200.0
    w = inputs.Workload(name="inertial", nx=4, ny=4, nz=3, periodic_x=True, periodic_y=True,
                        f0=f, beta=0.0, tau0=0.0, noise_std=0.0, dt=dt, chi=chi)
    inp = inputs.make_inputs(w)
    m = oracle.OracleModel.from_inputs(w, inp)
    shape = (w.nz, w.ny, w.nx)
    m.set("u", np.full(shape, 0.1))
    m.set("U", np.full((w.ny, w.nx), 0.1 * w.depth))
    # the substeps add the slow forcing linearly, U^l = U^n + l dtau G/dt, so the
    # window average is U^n + G (first moment Ns) and Ubar = U^n + c G with
    # c = sum_l A_l l / Ns^2 = sum_q a_q q (q - 1) / (2 Ns^2)
    q, a = _window(w.n_substeps)
    c = float(np.sum(a * q * (q - 1))) / (2.0 * w.n_substeps ** 2)
    zs = [0.1 + 0j]
    for n in range(100):
        Ub = m.get("U")
        m.step(1)
        Um_expect = Ub + c * (m.get("U") - Ub)
        assert np.max(np.abs(m.get("U_mean") - Um_expect)) <= 1e-12 * np.max(np.abs(Ub))
        u, v = m.get("u"), m.get("v")
        assert np.ptp(u) <= 1e-13 and np.ptp(v) <= 1e-13  # uniform up to round-off
        zs.append(complex(u[0, 0, 0], v[0, 0, 0]))
    a = -1j * f * dt
    A, B = 1.5 + chi, 0.5 + chi
    q, Q, pred = [zs[0]], zs[0], [zs[0]]
    for n in range(100):
        G = a * q[0] if n == 0 else a * (A * q[n] - B * q[n - 1])
        q.append(Q + c * G)
        Q = Q + G
        pred.append(q[-1])
    err = max(abs(x - y) for x, y in zip(zs, pred))
    assert err <= 1e-12 * abs(zs[0])
    # characteristic roots of q^{n+2} = (1 + c a A) q^{n+1} + ((1-c) a A - c a B) q^n - (1-c) a B q^{n-1}:
    # the dominant one fixes frequency and amplitude drift; the scheme stays neutral to O((f dt)^2)
    roots = np.roots([1.0, -(1.0 + c * a * A), -((1.0 - c) * a * A - c * a * B), (1.0 - c) * a * B])
    lam = roots[np.argmax(np.abs(roots))]
    assert abs(abs(zs[-1]) / abs(zs[-31]) - abs(lam) ** 30) < 1e-6
    th = f * dt
    assert abs(abs(lam) - 1.0) < th ** 2
    assert abs(-np.angle(lam) / th - 1.0) < th


def test_restart_is_bitwise():
    w = small_latlon(nx=24, ny=14, nz=5)
    inp = inputs.make_inputs(w)
    a = oracle.OracleModel.from_inputs(w, inp)
    a.step(3)
    saved = {n: a.get(n) for n in ("u", "v", "T", "eta", "U", "V", "gu_prev", "gv_prev", "gt_prev")}
    first = a.first_step
    a.step(3)
    b = oracle.OracleModel.from_inputs(w, inp)
    for n, arr in saved.items():
        b.set(n, arr)
    b.first_step = first
    b.step(3)
    for n in ("u", "v", "T", "eta", "U", "V", "eta_mean", "U_mean", "V_mean"):
        assert np.array_equal(a.get(n), b.get(n)), n


def test_long_run_stays_bounded():
    """A 1/4-degree regional box with seamounts, wind and restoring stays near
    rest for 40 hours (240 steps of 600 s): the wind-driven flow stays below a
    few cm/s and the free surface within centimetres. Correcting the depth
    mean with the end-of-substep transport instead of the substep average
    lets fast modes grow here (|u| > 2 m/s by step 240)."""
    from paper_2309_06662_amd import closure_train

    w, _ = closure_train.regional_pair(nx=32, ny=24, nz=10)
    m = oracle.OracleModel.from_inputs(w, inputs.make_inputs(w))
    m.step(240)
    d = m.diagnostics()
    assert d["nonfinite"] == 0
    assert d["max_abs_u"] < 0.2 and d["max_abs_v"] < 0.2
    assert max(abs(d["eta_min"]), abs(d["eta_max"])) < 0.1
