"""Parity at the full 1/12-degree size (4320 x 1800 x 100, the benchmarked
configuration), on sampled outputs the oracle can compute one by one.

One step moves information at most 3 cells through the tendency stencils (one
more through the velocity masks) and one cell per barotropic substep (60 at
this size), so after two steps a column depends only on the initial state
within 2 x 64 = 128 columns of it. The oracle steps a bounded window of
radius 134 columns cut from the seeded inputs, twice, and the centre 5 x 5
patch must match the GPU's state after its second step: FP64 within 1e-11
relative, FP32 within 1e-4. Both sides start from the same inputs; nothing
the GPU computed enters the oracle.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs

pytestmark = pytest.mark.gpu

R = 134     # window radius in columns
P = 2       # half-width of the compared patch
STEPS = 2
W = inputs.LATLON_TWELFTH
SAMPLES = [(100, 900), (2160, 300), (4300, 1500)]  # (i, j): equator-ish, southern ocean, near the x seam


def _window(ic, jc):
    cols = np.arange(ic - R, ic + R + 1) % W.nx
    j0, j1 = max(0, jc - R), min(W.ny, jc + R + 1)
    rows = np.arange(j0, j1)
    win = W.replace(name=f"window_{ic}_{jc}", nx=len(cols), ny=len(rows), periodic_x=False,
                    x0=W.x0 + (ic - R) * W.dx, y0=W.y0 + j0 * W.dy)
    sub = lambda a: a[..., rows[:, None], cols[None, :]]
    return win, sub, jc - j0


@functools.lru_cache(maxsize=None)
def _inputs():
    print(f"full-size {W.name}: inputs", flush=True)
    return inputs.make_inputs(W)


@functools.lru_cache(maxsize=None)
def _oracle_patch(ic, jc):
    """The oracle's fields on the centre patch after STEPS steps (shared by both precisions)."""
    inp = _inputs()
    win, sub, jcw = _window(ic, jc)
    print(f"  oracle window {win.nx}x{win.ny}x{win.nz} around ({ic},{jc})", flush=True)
    ref = oracle.OracleModel(win, inp["dz"], sub(inp["kbottom"]))
    ref.set("T", sub(inp["T0"]))
    for n in ("taux", "tauy", "tstar"):
        ref.set(n, sub(inp[n]))
    ref.step(STEPS)
    out = {n: ref.get(n)[..., jcw - P:jcw + P + 1, R - P:R + P + 1] for n in ("u", "v", "T", "eta", "U", "V")}
    ref.close()
    return out


def _check(precision, tol):
    from paper_2309_06662_amd import ocn

    inp = _inputs()
    gpu = ocn.Model(W, precision, inp)
    print(f"full-size {precision}: {STEPS} steps on the GPU", flush=True)
    gpu.step(STEPS)
    got_all = {n: gpu.get(n) for n in ("u", "v", "T", "eta", "U", "V")}
    del gpu
    worst = 0.0
    for ic, jc in SAMPLES:
        _, sub, jcw = _window(ic, jc)
        ref = _oracle_patch(ic, jc)
        for n, a in got_all.items():
            got = sub(a)[..., jcw - P:jcw + P + 1, R - P:R + P + 1]
            exp = ref[n]
            err = np.linalg.norm(got - exp) / max(np.linalg.norm(exp), 1e-300)
            worst = max(worst, err)
            print(f"  sample ({ic},{jc}) {n}: rel L2 {err:.2e}", flush=True)
            assert err <= tol, (ic, jc, n, err)
    assert np.isfinite(worst)


def test_fullsize_fp64_sampled_columns():
    _check("fp64", 1e-11)


def test_fullsize_fp32_sampled_columns():
    _check("fp32", 1e-4)
