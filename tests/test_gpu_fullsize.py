"""Parity at the full 1/12-degree size (4320 x 1800 x 100, the benchmarked
configuration), on sampled outputs the oracle can compute one by one.

One step moves information at most 3 cells through the tendency stencils and
one cell per barotropic substep (60 at this size), so a column's value after a
step depends only on the state within 63 columns of it. The oracle steps a
bounded window of radius 68 columns cut from the GPU's state (all levels,
AB2 history included) and the centre 5 x 5 patch must match the GPU's next
step: FP64 within 1e-11 relative, FP32 within 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs

pytestmark = pytest.mark.gpu

R = 68      # window radius in columns
P = 2       # half-width of the compared patch
W = inputs.LATLON_TWELFTH
SAMPLES = [(100, 900), (2160, 300), (4300, 1500)]  # (i, j): equator-ish, southern ocean, near the x seam


def _window(full, kb, inp, ic, jc):
    cols = np.arange(ic - R, ic + R + 1) % W.nx
    j0, j1 = max(0, jc - R), min(W.ny, jc + R + 1)
    rows = np.arange(j0, j1)
    win = W.replace(name=f"window_{ic}_{jc}", nx=len(cols), ny=len(rows), periodic_x=False,
                    x0=W.x0 + (ic - R) * W.dx, y0=W.y0 + j0 * W.dy)
    sub = lambda a: a[..., rows[:, None], cols[None, :]]
    return win, sub, jc - j0


def _check(precision, tol):
    from paper_2309_06662_amd import ocn

    print(f"full-size {W.name} {precision}: inputs", flush=True)
    inp = inputs.make_inputs(W)
    gpu = ocn.Model(W, precision, inp)
    gpu.step(1)
    names3 = ("u", "v", "T", "gu_prev", "gv_prev", "gt_prev")
    names2 = ("eta", "U", "V")
    s1 = {n: gpu.get(n) for n in names3 + names2}
    print(f"full-size {precision}: step 2 on the GPU", flush=True)
    gpu.step(1)
    s2 = {n: gpu.get(n) for n in ("u", "v", "T", "eta", "U", "V")}
    worst = 0.0
    for ic, jc in SAMPLES:
        win, sub, jcw = _window(None, inp["kbottom"], inp, ic, jc)
        ref = oracle.OracleModel(win, inp["dz"], sub(inp["kbottom"]))
        for n in ("taux", "tauy", "tstar"):
            ref.set(n, sub(inp[n]))
        for n, a in s1.items():
            ref.set(n, sub(a))
        ref.first_step = False
        ref.step(1)
        for n in ("u", "v", "T", "eta", "U", "V"):
            got = sub(s2[n])[..., jcw - P:jcw + P + 1, R - P:R + P + 1]
            exp = ref.get(n)[..., jcw - P:jcw + P + 1, R - P:R + P + 1]
            err = np.linalg.norm(got - exp) / max(np.linalg.norm(exp), 1e-300)
            worst = max(worst, err)
            print(f"  sample ({ic},{jc}) {n}: rel L2 {err:.2e}", flush=True)
            assert err <= tol, (ic, jc, n, err)
    assert np.isfinite(worst)


def test_fullsize_fp64_sampled_columns():
    _check("fp64", 1e-11)


def test_fullsize_fp32_sampled_columns():
    _check("fp32", 1e-4)
