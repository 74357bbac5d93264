"""Train the learned vertical-mixing closure on coarse-grained higher-resolution
runs, and evaluate it against the constant diffusivity.

The paper motivates learning unresolved processes from data (Sec. 3) and runs
with a vertical-mixing closure (Sec. 6). This module builds that data from the
library's own runs:

1. A regional box of the lat-lon basin (seamounts, cos-latitude wind, surface
   restoring) is run at a resolution `factor` times finer than the coarse
   target grid, same levels, with a mixing parameterization: convective
   adjustment (kappa_conv where N^2 < 0) or Richardson-number mixing (the
   library's Pacanowski-Philander reading, convective where N^2 < 0): surface
   cooling by the restoring makes the upper ocean statically unstable, and a
   hydrostatic model needs that mixing to stay well posed.
2. Every `sample_every` fine steps the fine state is coarse-grained onto the
   coarse grid (area-weighted means over wet fine cells; a coarse cell counts
   only where all its fine cells are wet). The subgrid heat flux through each
   coarse z-face is the eddy flux <w T> - <w><T> plus the fine model's mixing
   beyond the background, -<(kappa - kappa0) dT/dz>, averaged over a window of
   samples.
3. Target: kappa_eff = kappa0 + max(0, -F / D) for that subgrid flux F, with
   D = d<T>/dz kept at least 1e-6 K/m in magnitude with its sign (a
   down-gradient flux gives a positive diffusivity in stable and unstable
   stratification alike), clipped to [1e-6, 1] m^2/s, as log10 at layer centres
   (mean of the centre's wet faces; the background at dry levels). Inputs: the
   library's closure features of the coarse model set to the coarse-grained
   state, normalised over the training set.
4. The network (Linear-ReLU-Linear-ReLU-Linear, BF16 on the matrix cores,
   FP32 Adam) trains on the windows before the held-out period.
5. Evaluation, declared before any run: from the coarse-grained state at the
   start of the held-out period, the coarse model runs `eval_days` with the
   constant diffusivity (the baseline), with the trained network, and, as a
   physical comparator, with the fine run's mixing parameterization; against the
   coarse-grained truth at the end, the RMSE over valid columns of the
   mixed-layer depth (first depth where T falls 0.2 K below the top layer)
   and of the change in column heat content sum dz T are reported for both.
6. Optionally (basin_eval), the trained network runs on the whole 1/4-degree
   basin, whose grid spacing, levels and time step the training box shares,
   beside the constant diffusivity and the fine run's own parameterization,
   which stands in for a finer truth of the whole basin; the time per step of
   each run is the closure's cost with trained weights.

    python -m paper_2309_06662_amd.closure_train --out DIR [--days 20 --eval-days 4 ...]
"""
import argparse
import json
import math
import os
import time

import numpy as np

from . import inputs


def regional_pair(factor=4, nx=96, ny=64, nz=50, lon0=150.0, lat0=-60.0, res=0.25, depth=5500.0,
                  dt_coarse=600.0, n_substeps=60):
    """Coarse and fine workloads over the same box (bounded, seamount bathymetry, restoring)."""
    coarse = inputs.Workload(name=f"region_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, coords="latlon",
                             periodic_x=False, x0=lon0, y0=lat0, dx=res, dy=res, depth=depth,
                             bathymetry="seamounts", dt=dt_coarse, n_substeps=n_substeps, restore_days=30.0)
    fine = coarse.replace(name=f"region_{nx * factor}x{ny * factor}x{nz}", nx=nx * factor, ny=ny * factor,
                          dx=res / factor, dy=res / factor, dt=dt_coarse / factor)
    return coarse, fine


class CoarseGrainer:
    """Area-weighted means of fine fields over blocks of factor x factor columns."""

    def __init__(self, coarse, fine, kb_fine, kb_coarse, factor):
        self.f = factor
        self.nz = fine.nz
        lat = fine.y0 + (np.arange(fine.ny) + 0.5) * fine.dy
        self.area = np.repeat(np.cos(np.radians(lat))[:, None], fine.nx, axis=1)  # relative areas
        k = np.arange(fine.nz)[:, None, None]
        self.wet_f = k >= fine.nz - kb_fine[None]                   # [nz, NY, NX]
        wet_c = k >= coarse.nz - kb_coarse[None]                    # [nz, ny, nx]
        allwet = self._block(self.wet_f.astype(np.float64), weights=False) >= 1.0 - 1e-12
        self.valid = wet_c & allwet                                 # coarse cells fully resolved below
        # coarse ocean columns whose every wet cell is fully resolved by fine wet cells
        self.valid_col = (kb_coarse >= 2) & (self.valid == wet_c).all(axis=0)

    def _block(self, a, weights=True):
        f = self.f
        *lead, NY, NX = a.shape
        if weights:
            w = self.area
            num = (a * w).reshape(*lead, NY // f, f, NX // f, f).sum(axis=(-3, -1))
            den = np.broadcast_to(w, a.shape).reshape(*lead, NY // f, f, NX // f, f).sum(axis=(-3, -1))
            return num / den
        return a.reshape(*lead, NY // f, f, NX // f, f).mean(axis=(-3, -1))

    def cells(self, a):
        return self._block(a)

    def u_faces(self, u):
        """Coarse u on coarse west faces: mean of the fine u on the same face line."""
        f = self.f
        nz, NY, NX = u.shape
        return u[:, :, ::f].reshape(nz, NY // f, f, NX // f).mean(axis=2)

    def v_faces(self, v):
        f = self.f
        nz, NY, NX = v.shape
        return v[:, ::f, :].reshape(nz, NY // f, NX // f, f).mean(axis=3)


def eddy_flux(cg, T, W, kappa=None, kappa0=0.0, dz=None):
    """Upward subgrid heat flux on interior z-faces (slot k = face between layers
    k-1 and k), coarse grid: <w T> - <w><T>, plus -<(kappa - kappa0) dT/dz>
    when the fine face diffusivity is given."""
    nz = T.shape[0]
    Tf = np.zeros_like(T)
    Tf[1:] = 0.5 * (T[1:] + T[:-1])
    w = W[:nz]                       # faces 0..nz-1 (bottom face of each layer)
    wet_face = np.zeros_like(cg.wet_f)
    wet_face[1:] = cg.wet_f[1:] & cg.wet_f[:-1]
    wT = np.where(wet_face, w * Tf, 0.0)
    wm = np.where(wet_face, w, 0.0)
    Tm = np.where(wet_face, Tf, 0.0)
    flux = cg.cells(wT) - cg.cells(wm) * cg.cells(Tm)
    if kappa is not None:
        dzc = np.zeros(nz)
        dzc[1:] = 0.5 * (dz[1:] + dz[:-1])
        dTdz = np.zeros_like(T)
        dTdz[1:] = (T[1:] - T[:-1]) / dzc[1:, None, None]
        flux = flux + cg.cells(np.where(wet_face, -(kappa - kappa0) * dTdz, 0.0))
    return flux


def kappa_target(flux, Tc, dz, kappa0):
    """log10 of kappa_eff on z-faces (slot k = face between layers k-1 and k,
    slot 0 the background) from face subgrid fluxes and coarse T, [nz, ny, nx]."""
    nz = Tc.shape[0]
    dzc = np.zeros(nz)
    dzc[1:] = 0.5 * (dz[1:] + dz[:-1])
    kf = np.full_like(flux, kappa0)
    dTdz = np.zeros_like(flux)
    dTdz[1:] = (Tc[1:] - Tc[:-1]) / dzc[1:, None, None]
    # down-gradient flux in either stratification: the gradient keeps its sign,
    # its magnitude is kept away from zero
    g = dTdz[1:]
    den = np.where(g >= 0.0, 1.0, -1.0) * np.maximum(np.abs(g), 1e-6)
    kf[1:] = kappa0 + np.maximum(0.0, -flux[1:] / den)
    return np.log10(np.clip(kf, 1e-6, 1.0))


def mixed_layer_depth(T, dz, thresh=0.2):
    """Depth of the first layer centre (from the top) colder than the top layer by thresh, [ny, nx]."""
    nz = T.shape[0]
    depth_c = np.cumsum(dz[::-1]) - 0.5 * dz[::-1]     # centre depths from the top
    Tt = T[nz - 1]
    mld = np.full(Tt.shape, depth_c[-1])
    found = np.zeros(Tt.shape, bool)
    for q in range(1, nz):
        k = nz - 1 - q
        hit = (~found) & (T[k] < Tt - thresh)
        mld[hit] = depth_c[q]
        found |= hit
    return mld


def heat_content(T, dz):
    return np.tensordot(dz, T, axes=(0, 0))


def _log(msg):
    print(f"[closure] {msg}", flush=True)


def attach_mixing(model, mixing, convective):
    """The fine run's mixing parameterization on a model."""
    model.attach_closure()
    if mixing == "richardson":
        model.set_richardson(conv=convective)
    else:
        model.set_convective(convective)


def basin_eval(net, norm, mixing, convective, days, w=None, band=None):
    """The trained network on the whole 1/4-degree basin (1440 x 600 x 50, the
    training box's grid spacing, levels and time step), from the seeded
    initial state for `days`: FP32 runs with the constant diffusivity, with the
    network, and with the fine run's own mixing parameterization at this
    resolution. No finer truth of the whole basin is run; the physical
    parameterization stands in for it: the mixed-layer depth and column heat
    content of the constant and learned runs are compared with it (RMSE over
    ocean columns, and over the ocean columns of the latitude band `band` =
    (south, north) in degrees, the training box's), and each run's time per
    step is reported (the learned one is the closure's cost with trained
    weights)."""
    import torch

    from . import ocn

    w = inputs.LATLON_QUARTER if w is None else w
    inp = inputs.make_inputs(w)
    dz, ocean = inp["dz"], inp["kbottom"] > 0
    steps = int(round(days * 86400.0 / w.dt))
    out, T_end = {"workload": w.name, "days": days, "steps": steps, "comparator": mixing}, {}
    for mode in ("constant", "learned", mixing):
        m = ocn.Model(w, "fp32", inp)
        if mode == "learned":
            m.attach_closure(net, norm)
        elif mode == mixing:
            attach_mixing(m, mixing, convective)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        el = time.perf_counter() - t0
        T_end[mode] = m.get("T")
        d = m.diagnostics(allow_unstable=True)
        out[mode] = {"ms_per_step": el / steps * 1e3, "finite": d["nonfinite"] == 0}
        if mode != "constant":
            m.detach_closure()
        m.close()
        torch.cuda.empty_cache()
    ref = T_end[mixing]
    mld_ref, hc_ref = mixed_layer_depth(ref, dz), heat_content(ref, dz)
    lat = w.y0 + (np.arange(w.ny) + 0.5) * w.dy
    regions = {"": ocean}
    if band is not None:
        regions["_band"] = ocean & ((lat >= band[0]) & (lat <= band[1]))[:, None]
        out["band_deg"] = list(band)
    for mode in ("constant", "learned"):
        mld_err = mixed_layer_depth(T_end[mode], dz) - mld_ref
        hc_err = heat_content(T_end[mode], dz) - hc_ref
        for suffix, cols in regions.items():
            out[mode]["mld_rmse_vs_comparator_m" + suffix] = float(np.sqrt(np.mean(mld_err[cols] ** 2)))
            out[mode]["heat_content_rmse_vs_comparator_Km" + suffix] = float(np.sqrt(np.mean(hc_err[cols] ** 2)))
    out["comparator_mld_mean_m"] = float(np.mean(mld_ref[ocean]))
    _log(f"basin: {json.dumps(out)}")
    return out


def _box_samples(coarse, fine, factor, mixing, convective, days, eval_days, sample_hours, window_samples, din,
                 collect=True):
    """The fine run of one box. Returns its training pairs (features X and
    log10 kappa targets Y of the fully resolved coarse columns, for the
    windows before the held-out period; empty when collect is false), the
    coarse-grained states at the start and at the end of the held-out period,
    the coarse inputs and the coarse-grainer."""
    from . import ocn

    inp_c, inp_f = inputs.make_inputs(coarse), inputs.make_inputs(fine)
    dz = inp_c["dz"]
    cg = CoarseGrainer(coarse, fine, inp_f["kbottom"], inp_c["kbottom"], factor)
    nz = coarse.nz
    _log(f"box {coarse.x0:.1f}E {coarse.y0:.1f}N: coarse {coarse.nx}x{coarse.ny}x{nz}, fine {fine.nx}x{fine.ny}x{nz}, "
         f"{int(cg.valid_col.sum())} fully resolved coarse columns, mixing {mixing}, convective {convective}")
    mixed = mixing == "richardson" or convective > 0.0
    fm = ocn.Model(fine, "fp32", inp_f)
    if mixed:
        attach_mixing(fm, mixing, convective)
    cm = ocn.Model(coarse, "fp32", inp_c)   # holds coarse-grained states for the features

    steps_per_sample = max(1, int(round(sample_hours * 3600.0 / fine.dt)))
    n_samples = int(round(days * 24.0 / sample_hours))
    eval_start = int(round((days - eval_days) * 24.0 / sample_hours))

    def coarse_state():
        u, v, T = fm.get("u"), fm.get("v"), fm.get("T")
        W = fm.get("w")
        eta = fm.get("eta")
        kap = fm.get("kappa") if mixed else None
        flux = eddy_flux(cg, T, W, kap, fine.kappa, dz)
        return {"u": cg.u_faces(u), "v": cg.v_faces(v), "T": cg.cells(T), "eta": cg.cells(eta)}, flux

    X_list, Y_list, snaps = [], [], {}
    acc, start_state = None, None
    t0 = time.time()
    for s in range(1, n_samples + 1):
        fm.step(steps_per_sample)
        st, flux = coarse_state()
        if start_state is None:
            start_state = st
        acc = flux if acc is None else acc + flux
        if s % window_samples == 0:
            flux_w = acc / window_samples
            acc = None
            if collect and s <= eval_start:
                y = kappa_target(flux_w, start_state["T"], dz, coarse.kappa)
                kwet = np.zeros((nz, coarse.ny, coarse.nx), bool)           # wet interior faces
                kk = np.arange(nz)[:, None, None]
                kwet[1:] = (kk[1:] > nz - inp_c["kbottom"][None])
                y = np.where(kwet, y, math.log10(coarse.kappa))
                for n in ("u", "v", "T"):
                    cm.set(n, start_state[n])
                X = cm.closure_features(din).cpu().numpy()
                cols = cg.valid_col.reshape(-1)
                X_list.append(X[cols])
                Y_list.append(y.reshape(nz, -1).T[cols])
            start_state = None
        if s in (eval_start, n_samples):
            snaps[s] = st
        if s % 8 == 0:
            d = fm.diagnostics(allow_unstable=True)
            _log(f"fine sample {s}/{n_samples} ({s * steps_per_sample} steps, {time.time() - t0:.0f} s, "
                 f"max|w| {d['max_abs_w']:.2e}, T {d['t_min']:.2f}..{d['t_max']:.2f})")
            if d["nonfinite"]:
                raise RuntimeError("the fine run became non-finite")
    fm.close()
    cm.close()
    return X_list, Y_list, (snaps[eval_start], snaps[n_samples]), inp_c, cg


def _evaluate(coarse, inp_c, cg, snaps, net, norm, mixing, convective, eval_days):
    """From the coarse-grained state at the start of the held-out period, the
    coarse model with the constant diffusivity, with the network and with the
    fine run's parameterization; RMSE of the mixed-layer depth and of the
    change of column heat content against the coarse-grained truth at the
    end, over the fully resolved columns."""
    from . import ocn

    dz = inp_c["dz"]
    start, truth = snaps
    eval_steps = int(round(eval_days * 86400.0 / coarse.dt))
    mixed = mixing == "richardson" or convective > 0.0
    results = {}
    vc = cg.valid_col
    for mode in (("constant", "learned", mixing) if mixed else ("constant", "learned")):
        m = ocn.Model(coarse, "fp32", inp_c)
        for n_ in ("u", "v", "T", "eta"):
            m.set(n_, start[n_])
        m.set("U", np.tensordot(dz, start["u"], axes=(0, 0)))
        m.set("V", np.tensordot(dz, start["v"], axes=(0, 0)))
        if mode == "learned":
            m.attach_closure(net, norm)
        elif mode == mixing:
            attach_mixing(m, mixing, convective)
        m.step(eval_steps)
        T_end = m.get("T")
        d = m.diagnostics(allow_unstable=True)
        mld_err = mixed_layer_depth(T_end, dz) - mixed_layer_depth(truth["T"], dz)
        hc_err = (heat_content(T_end, dz) - heat_content(start["T"], dz)) - \
                 (heat_content(truth["T"], dz) - heat_content(start["T"], dz))
        results[mode] = {"mld_rmse_m": float(np.sqrt(np.mean(mld_err[vc] ** 2))),
                         "heat_content_drift_rmse_Km": float(np.sqrt(np.mean(hc_err[vc] ** 2))),
                         "finite": d["nonfinite"] == 0}
        if mode != "constant":
            m.detach_closure()
        m.close()
    truth_drift = heat_content(truth["T"], dz) - heat_content(start["T"], dz)
    results["truth_heat_content_drift_rms_Km"] = float(np.sqrt(np.mean(truth_drift[vc] ** 2)))
    results["truth_mld_mean_m"] = float(np.mean(mixed_layer_depth(truth["T"], dz)[vc]))
    return results


def run(out_dir, factor=4, days=20.0, eval_days=4.0, sample_hours=3.0, window_samples=2, epochs=60,
        batch=4096, lr=1e-3, hidden=128, seed=0, convective=1.0, coarse_kw=None, mixing="convective",
        basin_days=0.0, boxes=None, eval_box=None):
    """mixing: the fine run's parameterization, "convective" (kappa = convective where
    N^2 < 0) or "richardson" (Richardson-number mixing with its default constants).
    boxes: south-west corners (lon, lat in degrees) of the training boxes (default
    the one of coarse_kw, else 150E 60S); the first is also evaluated over its
    held-out period. eval_box: the corner of a box left out of training, whose
    own fine run is the truth of a second evaluation over the same period.
    basin_days > 0 adds basin_eval of the trained network over that many days."""
    if mixing not in ("convective", "richardson"):
        raise ValueError("mixing must be 'convective' or 'richardson'")
    import torch

    from . import ocn

    os.makedirs(out_dir, exist_ok=True)
    kw = dict(coarse_kw or {})
    if boxes is None:
        boxes = [(kw.pop("lon0", 150.0), kw.pop("lat0", -60.0))]
    else:
        kw.pop("lon0", None)
        kw.pop("lat0", None)
    pairs = [regional_pair(factor=factor, lon0=lo, lat0=la, **kw) for lo, la in boxes]
    coarse = pairs[0][0]
    nz = coarse.nz
    din = (4 * nz + 3 + 7) // 8 * 8
    args = (factor, mixing, convective, days, eval_days, sample_hours, window_samples, din)
    X_list, Y_list, first = [], [], None
    for c, f in pairs:
        xl, yl, snaps, inp_c, cg = _box_samples(c, f, *args)
        X_list += xl
        Y_list += yl
        if first is None:
            first = (c, inp_c, cg, snaps)
    held = None
    if eval_box is not None:
        c, f = regional_pair(factor=factor, lon0=eval_box[0], lat0=eval_box[1], **kw)
        _, _, snaps, inp_c, cg = _box_samples(c, f, *args, collect=False)
        held = (c, inp_c, cg, snaps)

    X = np.concatenate(X_list).astype(np.float64)
    Y = np.concatenate(Y_list).astype(np.float64)
    wet = X != 0
    mean = np.array([X[:, f][wet[:, f]].mean() if wet[:, f].any() else 0.0 for f in range(din)])
    std = np.array([X[:, f][wet[:, f]].std() if wet[:, f].any() else 1.0 for f in range(din)])
    std[~(std > 1e-12)] = 1.0
    Xn = np.where(wet, (X - mean) / std, 0.0).astype(np.float32)
    _log(f"training set: {len(Xn)} columns from {len(pairs)} boxes, target log10 kappa mean {Y.mean():.2f} "
         f"sd {Y.std():.2f}")

    rng = np.random.default_rng(seed)
    P = [rng.normal(size=(din, hidden)) * math.sqrt(2.0 / din), np.zeros(hidden),
         rng.normal(size=(hidden, hidden)) * math.sqrt(2.0 / hidden), np.zeros(hidden),
         rng.normal(size=(hidden, nz)) * math.sqrt(1.0 / hidden), np.full(nz, float(Y.mean()))]
    net = ocn.Mlp(din, hidden, hidden, nz, max_batch=max(batch, max(c.nx * c.ny for c, _ in pairs)))
    net.set_params(np.concatenate([p.reshape(-1) for p in P]).astype(np.float32))
    xd = torch.from_numpy(Xn).cuda()
    yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    n = len(Xn)
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = perm[b0:b0 + batch]
            loss = net.train_step(xd[idx].contiguous(), yd[idx].contiguous(), lr)
            tot += loss
            cnt += 1
        losses.append(tot / max(cnt, 1))
    _log(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f} over {epochs} epochs")
    # baseline loss of predicting log10(kappa0) everywhere, for scale
    base = 0.5 * float(np.mean((Y - math.log10(coarse.kappa)) ** 2))

    # ---- evaluation from the start of the held-out period ----
    norm = np.concatenate([mean, std]).astype(np.float32)
    c0, inp0, cg0, snaps0 = first
    ev = _evaluate(c0, inp0, cg0, snaps0, net, norm, mixing, convective, eval_days)
    report = {"coarse": coarse.name, "fine": pairs[0][1].name, "factor": factor, "days": days,
              "eval_days": eval_days, "mixing": mixing, "convective_kappa": convective,
              "boxes": [list(b) for b in boxes], "train_columns": int(n), "din": din, "hidden": hidden,
              "epochs": epochs, "loss_first": losses[0], "loss_last": losses[-1], "loss_constant_kappa": base,
              "truth_heat_content_drift_rms_Km": ev.pop("truth_heat_content_drift_rms_Km"),
              "truth_mld_mean_m": ev.pop("truth_mld_mean_m"), "eval": ev}
    if held is not None:
        report["eval_box"] = list(eval_box)
        report["eval_region"] = _evaluate(*held, net, norm, mixing, convective, eval_days)
        _log(f"held-out region: {json.dumps(report['eval_region'])}")
    if basin_days > 0:
        report["basin"] = basin_eval(net, norm, mixing, convective, basin_days,
                                     band=(coarse.y0, coarse.y0 + coarse.ny * coarse.dy))
    with open(os.path.join(out_dir, "closure_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    np.save(os.path.join(out_dir, "closure_params.npy"), net.get_params())
    np.save(os.path.join(out_dir, "closure_norm.npy"), norm)
    _log(json.dumps(report["eval"]))
    return report


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--factor", type=int, default=4)
    ap.add_argument("--days", type=float, default=20.0)
    ap.add_argument("--eval-days", type=float, default=4.0)
    ap.add_argument("--sample-hours", type=float, default=3.0)
    ap.add_argument("--window", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--nx", type=int, default=96)
    ap.add_argument("--ny", type=int, default=64)
    ap.add_argument("--nz", type=int, default=50)
    ap.add_argument("--convective", type=float, default=1.0, help="kappa where N^2 < 0 in the fine run (0: off)")
    ap.add_argument("--mixing", choices=("convective", "richardson"), default="convective",
                    help="the fine run's mixing parameterization")
    ap.add_argument("--basin-days", type=float, default=0.0,
                    help="also run the trained network on the whole 1/4-degree basin for this many days")
    a = ap.parse_args()
    run(a.out, factor=a.factor, days=a.days, eval_days=a.eval_days, sample_hours=a.sample_hours,
        window_samples=a.window, epochs=a.epochs, convective=a.convective,
        coarse_kw={"nx": a.nx, "ny": a.ny, "nz": a.nz}, mixing=a.mixing, basin_days=a.basin_days)


if __name__ == "__main__":
    main()
