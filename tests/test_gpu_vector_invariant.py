"""GPU parity of the vector-invariant momentum form (paper Sec. 5.2: WENO
momentum advection on curvilinear grids; the form is the oracle's reading,
pinned in its own tests): the HIP path through the C ABI against the oracle
on the same seeded inputs.

- ten full steps: FP64 within 1e-11 and FP32 within 1e-4 relative L2 on u, v, T,
  eta, U, V over wet points, on a periodic lat-lon basin with seamounts
  (several tendency tiles, ragged tails, corners touching land at many
  levels) and a closed beta-plane basin; with salinity as well;
- the tendency stage alone within 1e-12: u*, v*, the momentum histories and
  the barotropic slow forcing;
- with a variable vertical mixing: a prescribed diffusivity field, and
  Richardson-number mixing (its own viscosity for u and v) diagnosed every
  step from a sheared state, steps within the same bounds;
- small and shallow domains (one to four levels, fewer columns than a tile
  and than the stencil's reach, periodic or walled) from a random flow;
- graph replay is bitwise the eager run; ensembles refuse the form.
"""
import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, rel_l2, small_latlon

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "T", "eta", "U", "V")
CASES = {
    "latlon": lambda: small_latlon(nx=70, ny=38, nz=7, tau0=0.2, momentum_form="vector_invariant"),
    "beta": lambda: inputs.BETA_BASIN_64.replace(name="beta_47x35x7", nx=47, ny=35, nz=7,
                                                 momentum_form="vector_invariant"),
    "latlon_salinity": lambda: small_latlon(nx=52, ny=30, nz=6, tau0=0.2, salinity=True,
                                            momentum_form="vector_invariant"),
}


def _ocn():
    from paper_2309_06662_amd import ocn

    return ocn


def _masks(w, kb):
    wet, mu, mv = masks(w, kb)
    col = kb > 0
    return {"u": mu, "v": mv, "T": wet, "S": wet, "u_pred": mu, "v_pred": mv, "gu_prev": mu, "gv_prev": mv,
            "eta": col, "U": col, "V": col, "gU_slow": col, "gV_slow": col, "T_pred": wet, "gt_prev": wet}


def _compare(ref, gpu, w, kb, tol, names):
    mk = _masks(w, kb)
    errs = {}
    for n in names:
        a = gpu.get(n)
        assert np.all(np.isfinite(a)), n
        errs[n] = rel_l2(a, ref.get(n), mk[n])
    print("  ", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_steps_match_oracle(case, precision, tol):
    w = CASES[case]()
    inp = inputs.make_inputs(w)
    print(f"case {w.name} {precision} vector-invariant", flush=True)
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, precision, inp)
    ref.step(10)
    gpu.step(10)
    names = FIELDS + (("S",) if w.salinity else ())
    _compare(ref, gpu, w, inp["kbottom"], tol, names)


@pytest.mark.parametrize("case", ["latlon", "beta"])
@pytest.mark.parametrize("first", [False, True])
def test_tendency_stage(case, first):
    w = CASES[case]()
    inp = inputs.make_inputs(w)
    rng = np.random.default_rng(31)
    _, mu, mv = masks(w, inp["kbottom"])
    shape = (w.nz, w.ny, w.nx)
    f = {"u": np.where(mu, 0.1 * rng.standard_normal(shape), 0.0),
         "v": np.where(mv, 0.1 * rng.standard_normal(shape), 0.0),
         "T": inp["T0"] + 0.2 * rng.standard_normal(shape)}
    for n in ("gu_prev", "gv_prev", "gt_prev"):
        f[n] = 1e-6 * rng.standard_normal(shape)
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, "fp64", inp)
    for n, a in f.items():
        ref.set(n, a)
        gpu.set(n, a)
    ref.first_step = first
    gpu.first_step = first
    ref.run_stage(oracle.STAGE_TENDENCY)
    gpu.run_stage(_ocn().STAGE_TENDENCY)
    _compare(ref, gpu, w, inp["kbottom"], 1e-12,
             ("u_pred", "v_pred", "T_pred", "gu_prev", "gv_prev", "gU_slow", "gV_slow"))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
@pytest.mark.parametrize("mixing", ["prescribed", "richardson"])
def test_with_variable_mixing(mixing, precision, tol):
    w = CASES["latlon"]()
    inp = inputs.make_inputs(w)
    rng = np.random.default_rng(17)
    _, mu, mv = masks(w, inp["kbottom"])
    shape = (w.nz, w.ny, w.nx)
    # a sheared start, so that Richardson numbers fall below the critical value in places
    u0 = np.where(mu, 0.05 * rng.standard_normal(shape), 0.0)
    v0 = np.where(mv, 0.05 * rng.standard_normal(shape), 0.0)
    print(f"case {w.name} {precision} vector-invariant, {mixing} mixing", flush=True)
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, precision, inp)
    gpu.attach_closure()
    for m in (ref, gpu):
        m.set("u", u0)
        m.set("v", v0)
    if mixing == "prescribed":
        kw = 10 ** rng.uniform(-5, -2, size=shape)
        kw[0] = 0.0
        ref.set("kappa", kw)
        gpu.set("kappa", kw)
    else:
        ref.set_richardson()
        gpu.set_richardson()
    ref.step(6)
    gpu.step(6)
    _compare(ref, gpu, w, inp["kbottom"], tol, FIELDS)


@pytest.mark.parametrize("shape,periodic", [((9, 7, 1), True), ((12, 5, 2), True), ((4, 3, 3), True),
                                            ((2, 2, 4), True), ((7, 6, 2), False), ((3, 9, 3), False)])
def test_small_and_shallow_domains(shape, periodic):
    nx, ny, nz = shape
    w = inputs.Workload(name=f"tiny_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, periodic_x=periodic, periodic_y=periodic,
                        dx=30e3, dy=30e3, depth=200.0 * nz, f0=1e-4, beta=2e-11, dt=900.0, n_substeps=15,
                        momentum_form="vector_invariant")
    inp = inputs.make_inputs(w)
    rng = np.random.default_rng(nx * 100 + ny)
    _, mu, mv = masks(w, inp["kbottom"])
    u = np.where(mu, 0.1 * rng.normal(size=(nz, ny, nx)), 0.0)
    v = np.where(mv, 0.1 * rng.normal(size=(nz, ny, nx)), 0.0)
    print(f"case {w.name} fp64 vector-invariant, periodic {periodic}", flush=True)
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, "fp64", inp)
    for m in (ref, gpu):
        m.set("u", u)
        m.set("v", v)
    ref.step(3)
    gpu.step(3)
    _compare(ref, gpu, w, inp["kbottom"], 1e-11, FIELDS)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replay_bitwise(precision):
    import torch

    ocn = _ocn()
    w = CASES["beta"]()
    inp = inputs.make_inputs(w)
    side = torch.cuda.Stream()
    a = ocn.Model(w, precision, inp, stream=side)
    b = ocn.Model(w, precision, inp)
    for n, graph in [(1, False), (2, True), (1, False), (2, True)]:
        a.step(n, graph=graph)
        b.step(n)
        a.synchronize()
        b.synchronize()
        for name in FIELDS:
            assert np.array_equal(a.get(name), b.get(name)), (n, graph, name)
    torch.cuda.synchronize()


def test_ensembles_refuse_the_form():
    ocn = _ocn()
    w = CASES["beta"]()
    with pytest.raises(ocn.OcnError):
        ocn.Ensemble([w, w], "fp32")
