"""Pins of the oracle's WENO reconstruction against what the mathematics fixes.

Reading of the paper's "WENO reconstructions" (Sec. 5.2): fifth-order WENO-Z
with Jiang-Shu smoothness indicators, order reduced to WENO3 and to upwind at
land. Checks: exactness on quadratics (every candidate stencil is exact for
them, whatever the weights), the ENO property at a jump, mirror symmetry,
convergence of the linear weights on smooth data, fifth-order convergence of the
flux divergence, and the order-reduction fallbacks.
"""
import math

import numpy as np
import pytest

import oracle


def _cell_avg_poly(c, x):
    """Average over [x-1/2, x+1/2] of c0 + c1 x + c2 x^2."""
    c0, c1, c2 = c
    return c0 + c1 * x + c2 * (x * x + 1.0 / 12.0)


@pytest.mark.parametrize("coef", [(1.0, 0.0, 0.0), (0.3, -2.0, 0.0), (1.5, 0.7, -3.0), (-2.0, 5.0, 11.0)])
def test_weno5_exact_on_quadratics(coef):
    # cells centred at -2..2, face at +1/2 between c (x=0) and d (x=1)
    s = [_cell_avg_poly(coef, x) for x in (-2, -1, 0, 1, 2)]
    exact = coef[0] + coef[1] * 0.5 + coef[2] * 0.25
    got = oracle.weno5z(*s)
    assert abs(got - exact) <= 1e-13 * max(1.0, abs(exact))


def test_weno3_exact_on_lines():
    for c0, c1 in [(1.0, 2.0), (-3.0, 0.5), (0.0, -7.0)]:
        b, c, d = (c0 + c1 * x for x in (-1, 0, 1))
        assert abs(oracle.weno3(b, c, d) - (c0 + 0.5 * c1)) <= 1e-14 * max(1, abs(c0) + abs(c1))


def test_weno5_eno_property_at_jump():
    # data 0,0,0 | 1,1: only the left stencil is smooth, the face value stays near 0
    assert abs(oracle.weno5z(0.0, 0.0, 0.0, 1.0, 1.0)) < 1e-6
    # data 0,0 | 1,1,1 with the jump upwind of c: the right stencil wins, value near 1
    assert abs(oracle.weno5z(0.0, 0.0, 1.0, 1.0, 1.0) - 1.0) < 1e-6


def test_weno5_smooth_limit_is_linear_fifth_order_scheme():
    # On smooth data the weights tend to (1/10, 6/10, 3/10): the result tends to
    # the linear upwind-biased scheme (2a - 13b + 47c + 27d - 3e)/60.
    errs = []
    for h in (0.1, 0.05, 0.025):
        x = np.array([-2, -1, 0, 1, 2]) * h + 0.3
        s = (np.sin(x + h / 2) - np.sin(x - h / 2)) / h  # cell averages of cos
        lin = (2 * s[0] - 13 * s[1] + 47 * s[2] + 27 * s[3] - 3 * s[4]) / 60.0
        errs.append(abs(oracle.weno5z(*s) - lin))
    assert errs[2] < errs[0] / 20


def test_weno5_reflection():
    # WENO-Z is reflection-equivariant: reconstructing reversed data with the
    # roles of the ends swapped equals the original reconstruction mirrored,
    # checked through an odd function whose mirror is its negative
    rng = np.random.default_rng(3)
    for _ in range(50):
        s = rng.normal(size=5)
        assert oracle.weno5z(*s) == pytest.approx(-oracle.weno5z(*(-s)), rel=1e-15, abs=1e-300)
        # adding a constant shifts the face value by that constant
        assert oracle.weno5z(*(s + 3.0)) == pytest.approx(oracle.weno5z(*s) + 3.0, rel=1e-14)


def test_zflux_mirror_symmetry():
    # reversing the column and the sign of the transport mirrors the face fluxes
    rng = np.random.default_rng(7)
    n = 12
    phi = rng.normal(size=n)
    wet = np.ones(n, dtype=np.int32)
    wf = rng.normal(size=n + 1)
    f = oracle.column_zflux(phi, wet, wf)
    g = oracle.column_zflux(phi[::-1].copy(), wet, -wf[::-1].copy())
    assert np.allclose(f, -g[::-1], rtol=1e-15, atol=0)


def test_reconstruct_order_reduction():
    s = np.array([5.0, 1.0, 2.0, 4.0, 9.0])
    full = np.ones(5, dtype=np.int32)
    assert oracle.reconstruct(s, full) == oracle.weno5z(*s)
    for bad in (0, 4):
        ok = full.copy()
        ok[bad] = 0
        assert oracle.reconstruct(s, ok) == oracle.weno3(1.0, 2.0, 4.0)
    for bad in (1, 3):
        ok = full.copy()
        ok[bad] = 0
        assert oracle.reconstruct(s, ok) == 2.0


def _flux_divergence_order(n_list):
    """L1 error of the semi-discrete divergence of a periodic sine, unit speed."""
    errs = []
    for n in n_list:
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        avg = (np.cos(2 * np.pi * (x - h / 2)) - np.cos(2 * np.pi * (x + h / 2))) / (2 * np.pi * h)
        # exact cell average of -d/dx sin(2 pi x)
        exact = -(np.sin(2 * np.pi * (x + h / 2)) - np.sin(2 * np.pi * (x - h / 2))) / h
        face = np.array([oracle.weno5z(*(avg[(i - 3 + r) % n] for r in range(5))) for i in range(n)])
        # face[i] is at x_{i-1/2}; divergence of cell i = (face[i+1] - face[i]) / h
        div = -(np.roll(face, -1) - face) / h
        errs.append(np.mean(np.abs(div - exact)))
    return [math.log2(errs[q] / errs[q + 1]) for q in range(len(errs) - 1)], errs


def test_weno5_fifth_order_convergence():
    orders, _ = _flux_divergence_order([16, 32, 64, 128, 256])
    # asymptotic orders on the finer pairs
    assert min(orders[1:]) >= 4.8, orders


def _fit_avg_poly(vals, centres):
    """Polynomial whose averages over the unit cells at `centres` equal `vals`."""
    n = len(vals)
    # average over [x-1/2, x+1/2] of x^p = ((x+1/2)^{p+1} - (x-1/2)^{p+1}) / (p+1)
    A = np.array([[((x + 0.5) ** (p + 1) - (x - 0.5) ** (p + 1)) / (p + 1) for p in range(n)] for x in centres])
    coef = np.linalg.solve(A, vals)
    return np.polynomial.Polynomial(coef)


def _smoothness(poly):
    """Jiang-Shu indicator: sum over derivative orders l >= 1 of the integral of
    (d^l p / dx^l)^2 over the target cell [-1/2, 1/2] (unit spacing)."""
    total = 0.0
    d = poly
    for _ in range(poly.degree()):
        d = d.deriv()
        sq = (d * d).integ()
        total += sq(0.5) - sq(-0.5)
    return total


def _weno_from_definitions(s, order):
    """WENO-Z (order 5) or WENO-JS (order 3) face value built from the
    definitions: candidate polynomials fitted to cell averages, smoothness by
    the Jiang-Shu integrals, weights alpha_r = d_r (1 + (tau/(beta_r+eps))^2) for
    WENO-Z with tau = |beta_0 - beta_2|, alpha_r = d_r / (beta_r + eps)^2 for JS."""
    eps = 1e-8
    if order == 5:
        cells = [(-2, -1, 0), (-1, 0, 1), (0, 1, 2)]
        vals = [s[0:3], s[1:4], s[2:5]]
        dlin = [0.1, 0.6, 0.3]
    else:
        cells = [(-1, 0), (0, 1)]
        vals = [s[0:2], s[1:3]]
        dlin = [1.0 / 3.0, 2.0 / 3.0]
    polys = [_fit_avg_poly(np.array(v, dtype=float), c) for v, c in zip(vals, cells)]
    q = [p(0.5) for p in polys]
    beta = [_smoothness(p) for p in polys]
    if order == 5:
        tau = abs(beta[0] - beta[2])
        alpha = [d * (1.0 + (tau / (b + eps)) ** 2) for d, b in zip(dlin, beta)]
    else:
        alpha = [d / (b + eps) ** 2 for d, b in zip(dlin, beta)]
    return sum(a * qq for a, qq in zip(alpha, q)) / sum(alpha)


def test_weno_matches_definitions_on_rough_data():
    rng = np.random.default_rng(17)
    for scale in (1e-4, 1e-2, 1.0, 30.0):
        for _ in range(40):
            s = scale * rng.normal(size=5)
            ref5 = _weno_from_definitions(s, 5)
            assert oracle.weno5z(*s) == pytest.approx(ref5, rel=1e-9, abs=1e-12 * scale)
            ref3 = _weno_from_definitions(s[1:4], 3)
            assert oracle.weno3(*s[1:4]) == pytest.approx(ref3, rel=1e-9, abs=1e-12 * scale)
