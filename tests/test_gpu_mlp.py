"""The closure network's matrix-core kernels against the oracle.

The GPU rounds inputs, weights and hidden activations to BF16 and accumulates
in FP32; the oracle runs in FP64. The forward test gives the oracle the same
BF16-rounded inputs and weights, so what remains is the rounding of the hidden
activations (about 2^-9 relative each) and the accumulation order: relative L2
within 1e-2. A tighter layout check rebuilds the GPU's arithmetic layer by
layer with numpy (BF16 rounding between layers): any transposed fragment or
swapped lane mapping shows as an O(1) error there. Gradients compare within
3e-2 relative L2 per tensor (the output error is also rounded to BF16 before
the backward products). The Adam update is checked exactly against the
oracle's Adam applied to the GPU's own gradients.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SHAPES = [(208, 128, 128, 56, 3000),   # a 50-level column's features, ragged row count, split-K active
          (24, 16, 32, 8, 70),         # tiny: single tiles, K smaller than one stage
          (64, 64, 64, 64, 64)]        # exact tiles
# Inference runs on the fused kernel when din % 8 == 0, h1 and h2 are multiples of
# 32 up to 128, din <= 256 and dout <= 128; the second shape above takes the
# layer-by-layer GEMM path. Extra forward cases for the fused kernel's edges:
FORWARD_SHAPES = SHAPES + [
    (208, 128, 128, 50, 1000),   # the closure's 50-level network, 50 outputs (partial block), ragged tile
    (256, 96, 64, 128, 300),     # widest input, unequal hidden widths, full output blocks
    (8, 32, 32, 1, 5)]           # one input chunk, one output, fewer rows than a block


def bf16_round(a):
    """Round float64/float32 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _setup(din, h1, h2, dout, n, seed):
    import torch
    from paper_2309_06662_amd import ocn

    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, din))
    T = rng.normal(size=(n, dout))
    P = [rng.normal(size=(din, h1)) * np.sqrt(2.0 / din), rng.normal(size=h1) * 0.1,
         rng.normal(size=(h1, h2)) * np.sqrt(2.0 / h1), rng.normal(size=h2) * 0.1,
         rng.normal(size=(h2, dout)) * np.sqrt(1.0 / h2), rng.normal(size=dout) * 0.1]
    net = ocn.Mlp(din, h1, h2, dout, max_batch=max(n, 128))
    flat = np.concatenate([p.reshape(-1) for p in P]).astype(np.float32)
    net.set_params(flat)
    xd = torch.from_numpy(X.astype(np.float32)).cuda()
    td = torch.from_numpy(T.astype(np.float32)).cuda()
    return net, X, T, P, xd, td


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("shape", FORWARD_SHAPES)
def test_forward_matches_oracle(shape):
    din, h1, h2, dout, n = shape
    net, X, T, P, xd, td = _setup(din, h1, h2, dout, n, seed=1)
    y = net.forward(xd).cpu().numpy().astype(np.float64)
    Xb = bf16_round(X)
    Pb = [bf16_round(p) if p.ndim == 2 else p.astype(np.float32).astype(np.float64) for p in P]
    Y, _, _ = oracle.mlp_forward(Xb, *Pb)
    err = _rel(y, Y)
    print(f"forward {shape}: rel L2 vs oracle {err:.2e}", flush=True)
    assert err <= 1e-2
    # layer-by-layer rebuild of the BF16 pipeline: layout errors would be O(1)
    W1, b1, W2, b2, W3, b3 = Pb
    H1 = bf16_round(np.maximum(Xb @ W1 + b1, 0.0))
    H2 = bf16_round(np.maximum(H1 @ W2 + b2, 0.0))
    Ye = H2 @ W3 + b3
    err2 = _rel(y, Ye)
    print(f"forward {shape}: rel L2 vs BF16 rebuild {err2:.2e}", flush=True)
    assert err2 <= 2e-3


@pytest.mark.parametrize("shape", SHAPES)
def test_gradients_match_oracle(shape):
    din, h1, h2, dout, n = shape
    net, X, T, P, xd, td = _setup(din, h1, h2, dout, n, seed=2)
    loss, g = net.gradients(xd, td)
    Xb = bf16_round(X)
    Pb = [bf16_round(p) if p.ndim == 2 else p.astype(np.float32).astype(np.float64) for p in P]
    ref_loss, ref_g = oracle.mlp_backward(Xb, T.astype(np.float32).astype(np.float64), *Pb)
    print(f"gradients {shape}: loss gpu {loss:.6e} oracle {ref_loss:.6e}", flush=True)
    assert loss == pytest.approx(ref_loss, rel=1e-2)
    for name, got, exp in zip(("W1", "b1", "W2", "b2", "W3", "b3"), net.unpack(g), ref_g):
        err = _rel(got.astype(np.float64), exp)
        print(f"  d{name}: rel L2 {err:.2e}", flush=True)
        assert err <= 3e-2, (name, err)


def test_deterministic_and_adam_step():
    din, h1, h2, dout, n = SHAPES[0]
    net, X, T, P, xd, td = _setup(din, h1, h2, dout, n, seed=3)
    p0 = net.get_params()
    l1, g1 = net.gradients(xd, td)
    l2, g2 = net.gradients(xd, td)
    assert l1 == l2 and np.array_equal(g1, g2)  # split-K partials are summed in a fixed order
    lr = 1e-3
    net.train_step(xd, td, lr)
    p1 = net.get_params().astype(np.float64)
    p = p0.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    oracle.adam(p, g1.astype(np.float64), m, v, 1, lr=lr)
    assert np.max(np.abs(p1 - p)) <= 1e-6


def test_training_reduces_loss():
    """A fixed synthetic regression the network can represent: loss falls by 10x."""
    import torch
    from paper_2309_06662_amd import ocn

    rng = np.random.default_rng(4)
    din, h1, h2, dout, n = 32, 64, 64, 16, 2048
    X = rng.normal(size=(n, din))
    A = rng.normal(size=(din, dout)) / np.sqrt(din)
    T = np.tanh(X @ A)
    net = ocn.Mlp(din, h1, h2, dout, max_batch=n)
    P = [rng.normal(size=(din, h1)) * np.sqrt(2.0 / din), np.zeros(h1),
         rng.normal(size=(h1, h2)) * np.sqrt(2.0 / h1), np.zeros(h2),
         rng.normal(size=(h2, dout)) * np.sqrt(1.0 / h2), np.zeros(dout)]
    net.set_params(np.concatenate([p.reshape(-1) for p in P]).astype(np.float32))
    xd = torch.from_numpy(X.astype(np.float32)).cuda()
    td = torch.from_numpy(T.astype(np.float32)).cuda()
    first = net.train_step(xd, td, 3e-3)
    for _ in range(300):
        last = net.train_step(xd, td, 3e-3, want_loss=False)
    last = net.train_step(xd, td, 3e-3)
    print(f"training: loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.1 * first
