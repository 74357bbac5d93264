"""Pins of the oracle's closure network: the forward pass against numpy's
matrix products, the backward pass against central finite differences of the
loss, and Adam's first step against its closed form."""
import numpy as np
import pytest

import oracle


def _net(rng, din=13, h1=9, h2=7, dout=5, n=11):
    X = rng.normal(size=(n, din))
    W1, b1 = rng.normal(size=(din, h1)) / 3, rng.normal(size=h1) / 3
    W2, b2 = rng.normal(size=(h1, h2)) / 3, rng.normal(size=h2) / 3
    W3, b3 = rng.normal(size=(h2, dout)) / 3, rng.normal(size=dout) / 3
    T = rng.normal(size=(n, dout))
    return X, T, [W1, b1, W2, b2, W3, b3]


def test_forward_matches_numpy():
    rng = np.random.default_rng(0)
    X, _, P = _net(rng)
    W1, b1, W2, b2, W3, b3 = P
    Y, H1, H2 = oracle.mlp_forward(X, *P)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    assert np.allclose(H1, h1, rtol=1e-13, atol=1e-14)
    assert np.allclose(H2, h2, rtol=1e-13, atol=1e-14)
    assert np.allclose(Y, h2 @ W3 + b3, rtol=1e-12, atol=1e-13)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    X, T, P = _net(rng)
    loss, grads = oracle.mlp_backward(X, T, *P)
    Y, _, _ = oracle.mlp_forward(X, *P)
    assert loss == pytest.approx(0.5 * np.mean((Y - T) ** 2), rel=1e-13)
    h = 1e-6
    for p, g in zip(P, grads):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        for q in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            old = flat[q]
            flat[q] = old + h
            lp, _ = oracle.mlp_backward(X, T, *P)
            flat[q] = old - h
            lm, _ = oracle.mlp_backward(X, T, *P)
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, gflat[q])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    p0 = p.copy()
    oracle.adam(p, g, m, v, t=1, lr=1e-2, eps=1e-8)
    # first step: bias-corrected moments equal g and g^2, so p moves by lr g / (|g| + eps)
    assert np.allclose(p, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
