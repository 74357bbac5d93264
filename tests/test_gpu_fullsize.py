"""Parity and stability at the full sizes of the two lat-lon grids: 1/12 degree
(4320 x 1800 x 100, the benchmarked configuration) and 1/4 degree
(1440 x 600 x 50).

Parity on sampled outputs the oracle can compute one by one. One step moves
information at most 3 cells through the tendency stencils (one more through
the velocity masks) and one cell per barotropic substep (90 at both sizes: 60
substeps per step, run on to 3/2 of the step), so after two steps a column
depends only on the initial state within 2 x 94 = 188 columns of it. The
oracle steps a bounded window of radius 200 columns cut from the seeded inputs,
twice (the windows on parallel threads: the oracle runs outside the
interpreter lock), and the centre 25 x 25 patch must match the GPU's state
after its second step: FP64 within 1e-11 relative, FP32 within 1e-4. (On a
5 x 5 patch at 180E, 50S the barotropic V moves by 5e-12 between two oracle
builds that differ only in fused multiply-adds: a field-wide relative norm, as
the tolerance is defined, needs a patch wider than that rounding-sensitive
spot.) The samples include the high latitudes, where converging meridians
make the internal waves fastest relative to the grid, and a ridge crest with
land. Both sides start from the same inputs; nothing the GPU computed enters
the oracle.

The same check covers the variants at 1/12 degree (salinity with the
quadratic equation of state together with vector-invariant momentum
advection) on three of the samples.

Stability: 100 steps of the whole 1/12-degree grid and 200 of the 1/4-degree
grid stay finite with bounded velocities and free surface, in both precisions.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs

pytestmark = pytest.mark.gpu

R = 200     # window radius in columns
P = 12      # half-width of the compared patch (R - 2 x 94 = 12 columns stay clean)
STEPS = 2
TWELFTH = inputs.LATLON_TWELFTH
QUARTER = inputs.LATLON_QUARTER
# (i, j) per grid: equator-ish, southern ocean, near the x seam, 70S, a ridge crest with land
SAMPLES = {
    TWELFTH.name: [(100, 900), (2160, 300), (4300, 1500), (1800, 60), (1080, 900)],
    QUARTER.name: [(720, 30), (0, 412), (1100, 560)],
}
# grids by key: the two lat-lon workloads, and the 1/12-degree one with salinity
# and vector-invariant momentum
VARIANT = TWELFTH.name + "+salinity+vector_invariant"
GRIDS = {TWELFTH.name: TWELFTH, QUARTER.name: QUARTER,
         VARIANT: TWELFTH.replace(salinity=True, momentum_form="vector_invariant")}
SAMPLES[VARIANT] = [(2160, 300), (1800, 60), (1080, 900)]


def _window(W, ic, jc):
    cols = np.arange(ic - R, ic + R + 1) % W.nx
    j0, j1 = max(0, jc - R), min(W.ny, jc + R + 1)
    rows = np.arange(j0, j1)
    win = W.replace(name=f"window_{ic}_{jc}", nx=len(cols), ny=len(rows), periodic_x=False,
                    x0=W.x0 + (ic - R) * W.dx, y0=W.y0 + j0 * W.dy)
    sub = lambda a: a[..., rows[:, None], cols[None, :]]
    return win, sub, jc - j0


@functools.lru_cache(maxsize=2)
def _inputs(key):
    print(f"full-size {key}: inputs", flush=True)
    return inputs.make_inputs(GRIDS[key])


def _fields(W):
    return ("u", "v", "T", "eta", "U", "V") + (("S",) if W.salinity else ())


def _oracle_window(args):
    """The oracle on one window: its centre patch after STEPS steps."""
    win, dz, kb, fields, jcw = args
    ref = oracle.OracleModel(win, dz, kb)
    for n, a in fields.items():
        ref.set(n, a)
    ref.step(STEPS)
    out = {n: ref.get(n)[..., jcw - P:jcw + P + 1, R - P:R + P + 1] for n in _fields(win)}
    ref.close()
    return out


@functools.lru_cache(maxsize=None)
def _oracle_patches(key):
    """The oracle's centre patches of every sample of a grid (shared by both precisions)."""
    import concurrent.futures as cf

    W = GRIDS[key]
    inp = _inputs(key)
    jobs = []
    for ic, jc in SAMPLES[key]:
        win, sub, jcw = _window(W, ic, jc)
        print(f"  oracle window {win.nx}x{win.ny}x{win.nz} around ({ic},{jc})", flush=True)
        fields = {"T": sub(inp["T0"]), "taux": sub(inp["taux"]), "tauy": sub(inp["tauy"]), "tstar": sub(inp["tstar"])}
        if W.salinity:
            fields.update(S=sub(inp["S0"]), sstar=sub(inp["sstar"]))
        jobs.append((win, inp["dz"], sub(inp["kbottom"]), fields, jcw))
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        return dict(zip(SAMPLES[key], ex.map(_oracle_window, jobs)))


def _check(key, precision, tol):
    from paper_2309_06662_amd import ocn

    W = GRIDS[key]
    ref_all = _oracle_patches(key)
    inp = _inputs(key)
    gpu = ocn.Model(W, precision, inp)
    print(f"full-size {key} {precision}: {STEPS} steps on the GPU", flush=True)
    gpu.step(STEPS)
    got_all = {n: gpu.get(n) for n in _fields(W)}
    gpu.close()
    del gpu
    import torch

    torch.cuda.empty_cache()  # the next grid's arena is a different size
    worst = 0.0
    for ic, jc in SAMPLES[key]:
        _, sub, jcw = _window(W, ic, jc)
        ref = ref_all[(ic, jc)]
        for n, a in got_all.items():
            got = sub(a)[..., jcw - P:jcw + P + 1, R - P:R + P + 1]
            exp = ref[n]
            err = np.linalg.norm(got - exp) / max(np.linalg.norm(exp), 1e-300)
            worst = max(worst, err)
            print(f"  sample ({ic},{jc}) {n}: rel L2 {err:.2e}", flush=True)
            assert err <= tol, (ic, jc, n, err)
    assert np.isfinite(worst)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_fullsize_twelfth_sampled_columns(precision, tol):
    _check(TWELFTH.name, precision, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_fullsize_quarter_sampled_columns(precision, tol):
    _check(QUARTER.name, precision, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_fullsize_twelfth_variants_sampled_columns(precision, tol):
    _check(VARIANT, precision, tol)


@pytest.mark.parametrize("name,steps", [(TWELFTH.name, 100), (QUARTER.name, 200)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fullsize_long_run_stays_bounded(name, steps, precision):
    from paper_2309_06662_amd import ocn

    W = GRIDS[name]
    gpu = ocn.Model(W, precision, _inputs(name))
    for done in range(0, steps, 25):
        gpu.step(25)
        d = gpu.diagnostics(allow_unstable=True)
        print(f"  {name} {precision} step {done + 25}: max|u| {d['max_abs_u']:.3e} max|v| {d['max_abs_v']:.3e} "
              f"eta [{d['eta_min']:.3e}, {d['eta_max']:.3e}] cfl {d['cfl_adv']:.3f} nonfinite {d['nonfinite']}",
              flush=True)
        assert d["nonfinite"] == 0
        assert d["max_abs_u"] < 2.0 and d["max_abs_v"] < 2.0
        assert max(abs(d["eta_min"]), abs(d["eta_max"])) < 2.0
