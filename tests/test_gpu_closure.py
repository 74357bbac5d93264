"""GPU parity of the vertical-diffusivity closure against the oracle.

* Prescribed face diffusivity: the variable-coefficient column solve must
  match the oracle within 1e-11 (FP64) / 1e-4 (FP32) relative L2, like the
  constant-diffusivity path, on bounded, periodic and uneven-bathymetry grids.
* Features: the GPU's network inputs of a state the GPU and the oracle both
  reached from the same inputs; FP32 output, so 1e-6 relative per column.
* Output map: identical network outputs (including non-finite and clipped
  values) give the oracle's face field within 1e-14 (FP64) / 1e-6 (FP32).
* Network mode end to end: the oracle chain (oracle features, the network
  in the GPU's declared precision -- BF16 inputs, weights and hidden
  activations, wide accumulation -- the oracle's output map and the oracle's
  step) against the GPU's network inside its step. What remains is FP32
  versus FP64 accumulation in the products and the rare BF16 rounding tie it
  flips: one flip moves a hidden activation by one BF16 ulp (2^-8 relative),
  log10 kappa by up to about 1e-3 and kappa by up to about 0.3 percent, so
  kappa agrees within 1e-2 (a few flips) and the states, where diffusion is a
  small share of each step's change, within 1e-6 relative L2. The plain FP64
  network (no BF16 activations) stays within 5 percent in kappa.
"""
import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, rel_l2, small_latlon

pytestmark = pytest.mark.gpu


def _ocn():
    from paper_2309_06662_amd import ocn

    return ocn


def _random_kappa(w, seed):
    rng = np.random.default_rng(seed)
    kw = 10 ** rng.uniform(-5, -2, size=(w.nz, w.ny, w.nx))
    kw[0] = 0.0
    return kw


def _compare(ref, gpu, w, kb, tol, fields=("u", "v", "T", "eta", "U", "V")):
    wet, mu, mv = masks(w, kb)
    col = kb > 0
    mk = {"u": mu, "v": mv, "T": wet, "eta": col, "U": col, "V": col}
    errs = {n: rel_l2(gpu.get(n), ref.get(n), mk[n]) for n in fields}
    print("  rel L2:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    return errs


CASES = {
    "beta": lambda: (inputs.BETA_BASIN_64.replace(name="beta_70x40x8", nx=70, ny=40, nz=8), None),
    "latlon": lambda: (small_latlon(nx=100, ny=40, nz=8, dt=900.0, n_substeps=40), None),
    "steps_periodic": lambda: (inputs.BETA_BASIN_64.replace(name="steps_70x14x9", nx=70, ny=14, nz=9, depth=2700.0,
                                                            periodic_x=True, periodic_y=True, beta=0.0), 5),
    # deeper columns reach the other solver forms: 40 levels are register-resident in
    # FP32 and LDS-staged in FP64, 110 levels are LDS-staged in both
    "deep40": lambda: (inputs.BETA_BASIN_64.replace(name="beta_40x20x40", nx=40, ny=20, nz=40), 7),
    "deep110": lambda: (inputs.BETA_BASIN_64.replace(name="beta_24x16x110", nx=24, ny=16, nz=110), 8),
}


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", list(CASES))
def test_prescribed_kappa_matches_oracle(case, precision, tol):
    w, kb_seed = CASES[case]()
    inp = inputs.make_inputs(w)
    if kb_seed is not None:
        rng = np.random.default_rng(kb_seed)
        kb = rng.integers(0, w.nz + 1, size=(w.ny, w.nx)).astype(np.int32)
        kb[kb == 1] = 0
        inp["kbottom"] = kb
    print(f"case {case} {precision} {w.nx}x{w.ny}x{w.nz}", flush=True)
    kw = _random_kappa(w, 11)
    ref = oracle.OracleModel.from_inputs(w, inp)
    ref.set("kappa", kw)
    gpu = _ocn().Model(w, precision, inp)
    gpu.attach_closure()
    gpu.set("kappa", kw)
    assert np.allclose(gpu.get("kappa"), ref.get("kappa"), rtol=1e-6 if precision == "fp32" else 0, atol=0)
    ref.step(6)
    gpu.step(6)
    _compare(ref, gpu, w, inp["kbottom"], tol)


def test_detach_returns_to_constant_path():
    w = inputs.BETA_BASIN_64.replace(name="beta_40x30x6", nx=40, ny=30, nz=6)
    inp = inputs.make_inputs(w)
    a = _ocn().Model(w, "fp64", inp)
    b = _ocn().Model(w, "fp64", inp)
    b.attach_closure()            # initialised to the constant: same answer up to rounding of the two solvers
    a.step(3)
    b.step(3)
    for n in ("u", "v", "T"):
        assert rel_l2(b.get(n), a.get(n)) <= 1e-13
    b.detach_closure()
    a.step(2)
    b.step(2)
    assert rel_l2(b.get("T"), a.get("T")) <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_features_match_oracle(precision):
    w = small_latlon(nx=100, ny=40, nz=8, dt=900.0, n_substeps=40)
    inp = inputs.make_inputs(w)
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, precision, inp)
    ref.step(3)
    gpu.step(3)
    rng = np.random.default_rng(2)
    for din in (4 * w.nz + 3 + 5, 4 * w.nz + 3):  # padded, and the odd minimum width
        mean, std = rng.normal(size=din), rng.uniform(0.5, 2.0, size=din)
        for norm in (None, np.concatenate([mean, std])):
            X = gpu.closure_features(din, norm).cpu().numpy().astype(np.float64)
            E = ref.closure_features(din, *(None, None) if norm is None else (mean, std))
            err = np.linalg.norm(X - E, axis=1) / np.maximum(np.linalg.norm(E, axis=1), 1e-30)
            print(f"features {precision} din={din} norm={norm is not None}: max per-column rel {err.max():.2e}",
                  flush=True)
            assert err.max() <= (1e-6 if precision == "fp64" else 2e-5)
            assert np.array_equal(X == 0, E == 0) or precision == "fp32"


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-14), ("fp32", 1e-6)])
def test_kappa_map_matches_oracle(precision, tol):
    import torch

    w = inputs.BETA_BASIN_64.replace(name="steps_70x14x9", nx=70, ny=14, nz=9, depth=2700.0,
                                     periodic_x=True, periodic_y=False)
    inp = inputs.make_inputs(w)
    rng = np.random.default_rng(3)
    kb = rng.integers(0, w.nz + 1, size=(w.ny, w.nx)).astype(np.int32)
    inp["kbottom"] = kb
    ref = oracle.OracleModel.from_inputs(w, inp)
    gpu = _ocn().Model(w, precision, inp)
    gpu.attach_closure()
    ld = w.nz + 3
    Y = rng.uniform(-9.0, 1.5, size=(w.nx * w.ny, ld)).astype(np.float32)
    Y[rng.random(Y.shape) < 0.05] = np.nan
    Y[rng.random(Y.shape) < 0.02] = np.inf
    gpu.closure_kappa(torch.from_numpy(Y).cuda())
    got = gpu.get("kappa")
    exp = ref.closure_kappa(Y[:, :w.nz].astype(np.float64), w.kappa)
    assert np.all(got[0] == 0)
    nz_ = exp != 0
    assert np.array_equal(got != 0, nz_)
    assert np.max(np.abs(got[nz_] / exp[nz_] - 1.0)) <= tol


def _bf16(a):
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_network_closure_end_to_end():
    import torch

    ocn = _ocn()
    w = inputs.BETA_BASIN_64.replace(name="beta_shallow_48x40x8", nx=48, ny=40, nz=8, depth=800.0)
    inp = inputs.make_inputs(w)
    din = (4 * w.nz + 3 + 7) // 8 * 8
    h = 32
    rng = np.random.default_rng(7)
    P = [rng.normal(size=(din, h)) * np.sqrt(2.0 / din), rng.normal(size=h) * 0.1,
         rng.normal(size=(h, h)) * np.sqrt(2.0 / h), rng.normal(size=h) * 0.1,
         rng.normal(size=(h, w.nz)) * 0.3 / np.sqrt(h), np.full(w.nz, -2.0)]
    net = ocn.Mlp(din, h, h, w.nz, max_batch=w.nx * w.ny)
    net.set_params(np.concatenate([p.reshape(-1) for p in P]).astype(np.float32))
    Pb = [_bf16(p) if p.ndim == 2 else p.astype(np.float32).astype(np.float64) for p in P]

    ref = oracle.OracleModel.from_inputs(w, inp)
    X0 = ref.closure_features(din)
    wet = X0 != 0
    mean = np.array([X0[:, f][wet[:, f]].mean() if wet[:, f].any() else 0.0 for f in range(din)])
    std = np.array([X0[:, f][wet[:, f]].std() if wet[:, f].any() else 1.0 for f in range(din)])
    std[~(std > 1e-12)] = 1.0
    norm = np.concatenate([mean, std]).astype(np.float32)
    mean64, std64 = norm[:din].astype(np.float64), norm[din:].astype(np.float64)

    W1, b1, W2, b2, W3, b3 = Pb

    def bf16_network(X):
        H1 = _bf16(np.maximum(_bf16(X) @ W1 + b1, 0.0))
        H2 = _bf16(np.maximum(H1 @ W2 + b2, 0.0))
        return H2 @ W3 + b3

    gpu = ocn.Model(w, "fp64", inp)
    gpu.attach_closure(net, norm)
    for step in range(3):
        X = ref.closure_features(din, mean64, std64)
        kw = ref.closure_kappa(bf16_network(X), w.kappa)
        if step == 0:
            Yp, _, _ = oracle.mlp_forward(_bf16(X), *Pb)
            kp = ref.closure_kappa(Yp, w.kappa)
        ref.set("kappa", kw)
        ref.step(1)
        gpu.step(1)
        kg = gpu.get("kappa")
        m = kw != 0
        kerr = np.max(np.abs(kg[m] / kw[m] - 1.0))
        print(f"step {step + 1}: max kappa relative difference {kerr:.2e}", flush=True)
        assert kerr <= 1e-2
        if step == 0:
            perr = np.max(np.abs(kg[m] / kp[m] - 1.0))
            print(f"  vs the plain FP64 network: {perr:.2e}", flush=True)
            assert perr <= 0.05
    _compare(ref, gpu, w, inp["kbottom"], 1e-6)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_convective_adjustment_matches_oracle(precision, tol):
    """Convective adjustment (kappa_conv on faces with N^2 < 0, from the state
    at the start of each step) on a regional box whose top layer starts 10 K
    too cold in half of the columns."""
    from paper_2309_06662_amd import closure_train

    w, _ = closure_train.regional_pair(nx=40, ny=24, nz=10)
    inp = inputs.make_inputs(w)
    T0 = inp["T0"].copy()
    T0[-1, :, ::2] -= 10.0
    inp["T0"] = T0
    ref = oracle.OracleModel.from_inputs(w, inp)
    ref.set_convective(0.5)
    gpu = _ocn().Model(w, precision, inp)
    gpu.attach_closure()
    gpu.set_convective(0.5)
    ref.step(1)
    gpu.step(1)
    kr, kg = ref.get("kappa"), gpu.get("kappa")
    assert np.array_equal(kr == 0.5, np.isclose(kg, 0.5)), "unstable faces differ"
    assert (kr == 0.5).sum() > 0
    ref.step(19)
    gpu.step(19)
    _compare(ref, gpu, w, inp["kbottom"], tol)


RI_CASES = ["beta", "latlon", "steps_periodic", "deep40"]
_STATE_FIELDS = ("u", "v", "T", "eta", "U", "V", "gu_prev", "gv_prev", "gt_prev")


def _spun_up(case, steps=4):
    """The case after a few oracle steps, then given shear and a convective patch so
    every branch of the mixing formula occurs: currents alternating with depth
    (u +-0.15, v +-0.1 m/s between levels) over a tenth of the stratification
    (Ri from about 1e-2 up) and the top two layers of the western third 10 K
    colder (unstable faces)."""
    w, kb_seed = CASES[case]()
    inp = inputs.make_inputs(w)
    if kb_seed is not None:
        rng = np.random.default_rng(kb_seed)
        kb = rng.integers(0, w.nz + 1, size=(w.ny, w.nx)).astype(np.int32)
        kb[kb == 1] = 0
        inp["kbottom"] = kb
    ref = oracle.OracleModel.from_inputs(w, inp)
    ref.step(steps)
    sign = (-1.0) ** np.arange(w.nz)
    ref.set("u", ref.get("u") + 0.15 * sign[:, None, None])
    ref.set("v", ref.get("v") + 0.1 * sign[::-1, None, None])
    T = 10.0 + 0.1 * (ref.get("T") - 10.0)   # weaker stratification: Ri of order one
    T[-2:, :, : max(1, w.nx // 3)] -= 10.0
    ref.set("T", T)
    return w, inp, ref


def _copy_state(ref, gpu):
    for n in _STATE_FIELDS:
        gpu.set(n, ref.get(n))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", RI_CASES)
def test_richardson_faces_match_oracle(case, precision, tol):
    """The diagnosis alone, on the same state: the oracle's state is copied in."""
    w, inp, ref = _spun_up(case)
    gpu = _ocn().Model(w, precision, inp)
    _copy_state(ref, gpu)
    gpu.attach_closure()
    ref.set_richardson()
    gpu.set_richardson()
    nu_ref = ref.get("visc")
    wet = nu_ref != 0
    assert np.any(nu_ref == 1.0)                                   # convective faces occur
    assert np.any((nu_ref > 2e-4) & (nu_ref < 5e-3))               # intermediate Ri occurs
    for name in ("kappa", "visc"):
        got, exp = gpu.get(name), ref.get(name)
        assert np.array_equal(got == 0, exp == 0), name
        conv = exp == 1.0
        assert np.array_equal(got == 1.0, conv), name          # the same convective faces
        nz_ = exp != 0
        if precision == "fp64":
            err = np.max(np.abs(got[nz_] / exp[nz_] - 1.0))
        else:
            err = np.linalg.norm(got[nz_] - exp[nz_]) / np.linalg.norm(exp[nz_])
        print(f"{case} {precision} {name}: err {err:.2e}; convective faces {int(conv.sum())} of "
              f"{int(wet.sum())}, range {exp[nz_].min():.2e}..{exp[nz_].max():.2e}", flush=True)
        assert err <= tol, (name, err)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", RI_CASES)
def test_richardson_run_matches_oracle(case, precision, tol):
    """Six steps with the mixing diagnosed every step, from the perturbed state."""
    w, inp, ref = _spun_up(case, steps=2)
    gpu = _ocn().Model(w, precision, inp)
    _copy_state(ref, gpu)
    gpu.first_step = ref.first_step
    gpu.attach_closure()
    ref.set_richardson()
    gpu.set_richardson()
    ref.step(6)
    gpu.step(6)
    print(f"case {case} {precision} {w.nx}x{w.ny}x{w.nz}", flush=True)
    _compare(ref, gpu, w, inp["kbottom"], tol)
    err = rel_l2(gpu.get("visc"), ref.get("visc"))
    print(f"  visc rel L2 {err:.2e}", flush=True)
    assert err <= (1e-9 if precision == "fp64" else 1e-3)


def test_richardson_modes_and_errors():
    """Error codes of ocn_closure_richardson and the mode switches: convective
    adjustment replaces it (momentum back on the diffusivity), nu0 <= 0 sets every
    face back to the constant, detaching clears it."""
    ocn = _ocn()
    w = inputs.BETA_BASIN_64.replace(name="beta_24x20x6", nx=24, ny=20, nz=6)
    inp = inputs.make_inputs(w)
    m = ocn.Model(w, "fp64", inp)
    with pytest.raises(ocn.OcnError) as e:
        m.set_richardson()                      # no closure attached
    assert e.value.code == ocn.OCN_E_STATE
    m.attach_closure()
    for bad in (dict(alpha=-1.0), dict(nu_b=float("nan")), dict(conv=-0.5), dict(nu0=float("inf"))):
        with pytest.raises(ocn.OcnError) as e:
            m.set_richardson(**bad)
        assert e.value.code == ocn.OCN_E_INVALID, bad
    m.set_richardson()
    kap, nu = m.get("kappa"), m.get("visc")
    wet = kap != 0
    assert np.all(nu[wet] >= 1e-4) and np.all(kap[wet] >= 1e-5) and not np.array_equal(kap, nu)
    m.step(2)
    m.set_convective(1.0)                        # replaces Richardson mixing
    m.step(1)
    assert np.array_equal(m.get("visc"), m.get("kappa"))
    m.set_richardson()
    m.set_richardson(nu0=0.0)                    # off: the constant on every wet face
    assert np.all(m.get("kappa")[wet] == w.kappa) and np.array_equal(m.get("visc"), m.get("kappa"))
    m.set_richardson()
    m.detach_closure()
    assert np.all(m.get("visc")[wet] == w.kappa)
    m.step(1)
    assert m.diagnostics()["nonfinite"] == 0
