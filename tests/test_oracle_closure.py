"""Pins of the oracle's learned-closure plumbing: a prescribed face
diffusivity in the implicit vertical diffusion (checked against a dense
backward-Euler solve built from its definition), the per-column feature vector
on states with closed-form features, and the output -> diffusivity map."""
import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs


def _column_workload(nx, nz, **kw):
    base = dict(name="column", nx=nx, ny=1, nz=nz, coords="cartesian", periodic_x=True, periodic_y=True,
                dx=10e3, dy=10e3, depth=1000.0, f0=0.0, beta=0.0, dt=3600.0, n_substeps=10,
                restore_days=0.0, kappa=1e-3)
    base.update(kw)
    return inputs.BETA_BASIN_64.replace(**base)


def _dense_backward_euler(phi, dz, kface, dt):
    """(diag(dz) - dt L) x = dz phi with zero-flux ends; kface[k] sits between layers k-1 and k."""
    nz = len(phi)
    A = np.diag(dz.astype(float))
    for k in range(1, nz):
        g = dt * kface[k] / (0.5 * (dz[k - 1] + dz[k]))
        A[k, k] += g
        A[k - 1, k - 1] += g
        A[k, k - 1] -= g
        A[k - 1, k] -= g
    return np.linalg.solve(A, dz * phi)


def test_prescribed_kappa_equal_to_constant_is_the_constant_path():
    w = inputs.BETA_BASIN_64.replace(nx=12, ny=10, nz=6)
    inp = inputs.make_inputs(w)
    a = oracle.OracleModel.from_inputs(w, inp)
    b = oracle.OracleModel.from_inputs(w, inp)
    b.set("kappa", np.full((w.nz, w.ny, w.nx), w.kappa))
    a.step(3)
    b.step(3)
    for n in ("u", "v", "T", "eta"):
        assert np.array_equal(a.get(n), b.get(n)), n
    b.set("kappa", None)
    assert np.array_equal(b.get("kappa"), a.get("kappa"))


def test_prescribed_kappa_matches_dense_solve_for_tracer_and_momentum():
    """Two periodic columns at rest horizontally: only vertical diffusion acts.
    T diffuses with its own column's faces, u with the mean of the two columns."""
    nz = 7
    w = _column_workload(2, nz)
    dz = np.array([180.0, 160.0, 150.0, 140.0, 130.0, 120.0, 80.0])
    kb = np.full((1, 2), nz, dtype=np.int32)
    m = oracle.OracleModel(w, dz, kb)
    rng = np.random.default_rng(5)
    Tcol = 5.0 + rng.normal(size=nz)
    T = np.repeat(Tcol[:, None, None], 2, axis=2)
    ucol = rng.normal(size=nz) * 0.1
    u = np.repeat(ucol[:, None, None], 2, axis=2)
    kface = np.zeros((nz, 1, 2))
    kface[1:, 0, :] = 10 ** rng.uniform(-4, -1, size=(nz - 1, 2))
    m.set("T", T)
    m.set("u", u)
    m.set("U", np.full((1, 2), np.sum(dz * ucol)))
    m.set("kappa", kface)
    m.step(1)
    for i in range(2):
        exp_T = _dense_backward_euler(Tcol, dz, kface[:, 0, i], w.dt)
        assert np.allclose(m.get("T")[:, 0, i], exp_T, rtol=0, atol=1e-12)
    ku = 0.5 * (kface[:, 0, 0] + kface[:, 0, 1])  # u at i sits between the two columns (periodic)
    exp_u = _dense_backward_euler(ucol, dz, ku, w.dt)
    for i in range(2):
        assert np.allclose(m.get("u")[:, 0, i], exp_u, rtol=0, atol=1e-13)
    # the tracer-face field in use is the prescribed one on wet faces
    got = m.get("kappa")
    assert np.array_equal(got[1:], kface[1:]) and np.all(got[0] == 0)


def test_features_of_closed_form_state():
    nx, ny, nz = 5, 4, 6
    w = _column_workload(nx, nz, ny=ny, restore_days=10.0)
    dz = np.full(nz, 100.0)
    kb = np.full((ny, nx), nz, dtype=np.int32)
    kb[2, 3] = 0          # one land column
    kb[1, 1] = 3          # one shallow column
    m = oracle.OracleModel(w, dz, kb)
    z = np.cumsum(dz) - dz.sum() - 0.5 * dz
    T = np.broadcast_to((10.0 + 0.004 * z)[:, None, None], (nz, ny, nx)).copy()   # dT/dz = 0.004 K/m
    m.set("T", T)
    din = 4 * nz + 3 + 5
    m.set("taux", np.full((ny, nx), 0.07))
    m.set("tauy", np.full((ny, nx), -0.02))
    tstar = np.full((ny, nx), 7.0)
    m.set("tstar", tstar)
    X = m.closure_features(din)
    assert X.shape == (ny * nx, din)
    N2 = w.g * w.alpha * 0.004
    for j in range(ny):
        for i in range(nx):
            x = X[j * nx + i]
            K = kb[j, i]
            if K == 0:
                assert np.all(x == 0)
                continue
            wet = np.arange(nz) >= nz - K
            assert np.allclose(x[:nz][wet], T[wet, j, i], rtol=1e-15)
            assert np.all(x[:nz][~wet] == 0)
            assert np.all(x[nz:3 * nz] == 0)                     # fluid at rest
            n2 = x[3 * nz:4 * nz]
            face_wet = np.zeros(nz, bool)
            face_wet[1:] = wet[1:] & wet[:-1]
            assert np.allclose(n2[face_wet], N2, rtol=1e-12)
            assert np.all(n2[~face_wet] == 0)
            assert x[4 * nz] == pytest.approx(0.07) and x[4 * nz + 1] == pytest.approx(-0.02)
            q = 100.0 * (7.0 - T[nz - 1, j, i]) / (10.0 * 86400.0)
            assert x[4 * nz + 2] == pytest.approx(q, rel=1e-14)
            assert np.all(x[4 * nz + 3:] == 0)
    # normalisation applies to wet entries only
    rng = np.random.default_rng(0)
    mean, std = rng.normal(size=din), rng.uniform(0.5, 2.0, size=din)
    Xn = m.closure_features(din, mean, std)
    wet_entries = X != 0
    assert np.allclose(Xn[wet_entries], ((X - mean) / std)[wet_entries], rtol=1e-14)


def test_features_average_velocities_to_centres():
    nx, ny, nz = 6, 5, 3
    w = _column_workload(nx, nz, ny=ny)
    m = oracle.OracleModel(w, np.full(nz, 100.0), np.full((ny, nx), nz, dtype=np.int32))
    rng = np.random.default_rng(1)
    u, v = rng.normal(size=(nz, ny, nx)), rng.normal(size=(nz, ny, nx))
    m.set("u", u)
    m.set("v", v)
    X = m.closure_features(4 * nz + 3)
    uc = 0.5 * (u + np.roll(u, -1, axis=2))   # periodic in x and y
    vc = 0.5 * (v + np.roll(v, -1, axis=1))
    for j in range(ny):
        for i in range(nx):
            assert np.allclose(X[j * nx + i, nz:2 * nz], uc[:, j, i], rtol=1e-15)
            assert np.allclose(X[j * nx + i, 2 * nz:3 * nz], vc[:, j, i], rtol=1e-15)


def test_kappa_map():
    nx, nz = 4, 5
    w = _column_workload(nx, nz)
    kb = np.array([[5, 2, 0, 5]], dtype=np.int32)
    m = oracle.OracleModel(w, np.full(nz, 100.0), kb)
    Y = np.full((nx, nz), -3.0)
    Y[3] = [7.0, 2.0, -9.0, np.nan, -2.0]      # slot 0 (bottom face) is never used
    kw = m.closure_kappa(Y, kappa0=1e-5)
    assert np.all(kw[0] == 0)
    assert np.allclose(kw[1:, 0, 0], 1e-3, rtol=1e-14)
    assert np.allclose(kw[4, 0, 1], 1e-3, rtol=1e-14) and np.all(kw[:4, 0, 1] == 0)   # K = 2: one wet face
    assert np.all(kw[:, 0, 2] == 0)
    assert np.allclose(kw[1:, 0, 3], [1.0, 1e-7, 1e-5, 1e-2], rtol=1e-13)   # clipped, clipped, kappa0, plain


def test_convective_adjustment_mixes_unstable_faces_only():
    """A column with dense (cold) water over light water mixes those faces with
    kappa_conv; stable faces keep the constant: one step equals the dense
    backward-Euler solve with that face field, and the field follows T."""
    nz = 6
    w = _column_workload(1, nz, kappa=1e-5)
    dz = np.full(nz, 50.0)
    m = oracle.OracleModel(w, dz, np.full((1, 1), nz, dtype=np.int32))
    Tcol = np.array([4.0, 5.0, 6.0, 5.5, 7.0, 6.0])   # bottom first: faces 3 and 5 unstable
    m.set("T", Tcol[:, None, None])
    m.set_convective(0.5)
    m.step(1)
    kf = np.array([0.0, 1e-5, 1e-5, 0.5, 1e-5, 0.5])
    exp = _dense_backward_euler(Tcol, dz, kf, w.dt)
    assert np.allclose(m.get("T")[:, 0, 0], exp, rtol=0, atol=1e-12)
    assert np.array_equal(m.get("kappa")[:, 0, 0], kf)
    m.set_convective(0.0)
    assert np.all(m.get("kappa")[1:, 0, 0] == 1e-5)


# --- Richardson-number mixing (Pacanowski-Philander form; constants of the reading:
# nu0 = 1e-2, alpha = 5, nu_b = 1e-4, kappa_b = 1e-5, conv = 1 m^2/s) ---

def _richardson_column():
    """Two periodic columns, uniform in x, 100 m layers. Faces (k between layers k-1, k):
    1: no stratification, shear 0.1 m/s per 100 m      -> Ri = 0
    2: shear 0.1 m/s per 100 m, N^2 = 0.2 S^2          -> Ri = 1/alpha
    3: 0.5 K colder above                              -> convective
    4: 0.5 K warmer above, no shear                    -> Ri huge (background)"""
    nz = 5
    w = _column_workload(2, nz, kappa=1e-5)
    dz = np.full(nz, 100.0)
    m = oracle.OracleModel(w, dz, np.full((1, 2), nz, dtype=np.int32))
    s2 = (0.1 / 100.0) ** 2
    dT2 = 0.2 * s2 * 100.0 / (w.g * w.alpha)        # N^2 = g alpha dT / dzc = 0.2 S^2
    Tcol = np.array([10.0, 10.0, 10.0 + dT2, 9.5 + dT2, 10.0 + dT2])
    ucol = np.array([0.0, 0.1, 0.2, 0.5, 0.5])
    m.set("T", np.repeat(Tcol[:, None, None], 2, axis=2))
    m.set("u", np.repeat(ucol[:, None, None], 2, axis=2))
    m.set("U", np.full((1, 2), np.sum(dz * ucol)))
    return m, w, dz, Tcol, ucol


def test_richardson_faces_worked_values():
    m, w, dz, Tcol, ucol = _richardson_column()
    m.set_richardson()
    kap, nu = m.get("kappa")[:, 0, 0], m.get("visc")[:, 0, 0]
    # worked by hand from nu = nu0 r^2 + nu_b, kappa = nu r + kappa_b, r = 1 / (1 + 5 Ri)
    exp_nu = [0.0, 1.01e-2, 2.6e-3, 1.0, 1e-4]        # Ri = 0: nu0 + nu_b; Ri = 1/5: nu0/4 + nu_b
    exp_kap = [0.0, 1.011e-2, 1.31e-3, 1.0, 1e-5]     # Ri = 0: nu + kappa_b; Ri = 1/5: nu/2 + kappa_b
    assert np.allclose(nu[:4], exp_nu[:4], rtol=1e-12, atol=0)
    assert np.allclose(kap[:4], exp_kap[:4], rtol=1e-12, atol=0)
    assert abs(nu[4] - 1e-4) < 1e-15 and abs(kap[4] - 1e-5) < 1e-15   # r ~ 1e-13 on face 4
    assert np.array_equal(m.get("kappa")[:, 0, 0], m.get("kappa")[:, 0, 1])


def test_richardson_mixing_solves_tracer_with_kappa_and_momentum_with_viscosity():
    """At rest horizontally only vertical diffusion acts: T takes the diagnosed
    diffusivity, u the diagnosed viscosity (mean of the two identical columns)."""
    m, w, dz, Tcol, ucol = _richardson_column()
    m.set_richardson()
    kap, nu = m.get("kappa")[:, 0, 0].copy(), m.get("visc")[:, 0, 0].copy()
    m.step(1)   # diagnoses again from the same state, then steps
    assert np.allclose(m.get("T")[:, 0, 0], _dense_backward_euler(Tcol, dz, kap, w.dt), rtol=0, atol=1e-12)
    assert np.allclose(m.get("u")[:, 0, 1], _dense_backward_euler(ucol, dz, nu, w.dt), rtol=0, atol=1e-13)


def test_richardson_mode_switches():
    m, w, dz, Tcol, ucol = _richardson_column()
    m.set_richardson()
    assert not np.array_equal(m.get("visc"), m.get("kappa"))
    m.set_convective(1.0)      # convective adjustment replaces it: momentum uses the diffusivity again
    m.step(1)
    assert np.array_equal(m.get("visc"), m.get("kappa"))
    m.set_richardson(nu0=0.0)  # off: back to the constant
    assert np.all(m.get("kappa")[1:] == w.kappa) and np.all(m.get("visc")[1:] == w.kappa)
