#!/usr/bin/env python
"""Throughput of the split-explicit ocean step on one MI355X.

Metric: cell-updates per second (all interior cells, land included, per step)
and simulated years per day, at 1/12 degree (4320 x 1800 x 100, one GPU's
share of the paper's 1/48-degree runs), FP32 bulk arithmetic (the reported
value) and FP64 beside it, with the achieved fraction of the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample of the same
workload.

Inputs are synthetic and seeded (paper Sec. 6 forcing and bathymetry are not
available): see paper_2309_06662_amd/inputs.py. Every input is resident in HBM
before the timed region starts; the timed region is K whole steps (tendency +
AB2, barotropic substeps, column solve + correction), bracketed by device
synchronisation.

Beside the headline legs: the same grid with salinity and the quadratic
equation of state, and with vector-invariant momentum advection (FP32 each);
a 64-member ensemble of uneven basins; a small basin under graph replay; the
1/4-degree basin in both precisions, with the learned closure and with
Richardson-number mixing. Every leg reports whether its state stayed finite
and its largest speed; the run exits with status 3 when the headline leg
ended non-finite.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]

Counter tooling (for the traffic records under profiles/):
  python bench.py --copy-probe [--mib N]      a plain device copy of known size,
                                              to calibrate FETCH_SIZE / WRITE_SIZE
  python bench.py --stats-summary --stats-dir D --out F
                                              kernel table of a --kernel-trace --stats run
  python bench.py --sq-summary --sq1 A --sq2 B --out F
                                              SQ counter summary (VALU busy, instructions
                                              per cell) of two counter passes
  python bench.py --pmc-summary ...           per-launch HBM bytes of a kernel from
                                              two counter runs, scaled by the copy's
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2309_06662_amd import inputs, metrics  # noqa: E402

METRIC = "cell-updates/s & SYPD at 1/12° on 1 GPU, FP32 vs FP64; % of HBM roofline"

# Published MI355X peaks.
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

# Algorithmic work of the fused tendency + AB2 kernel per cell.
# Bytes: read u, v, T, G^{n-1} x3 and write u*, v*, T*, G^n x3 = 12 words.
TEND_WORDS_PER_CELL = 12
# Flops: 9 WENO-Z face reconstructions (three per advected field: x, y, z)
# at 74 operations each (17 candidate values, 18 differences, 15 smoothness
# indicators, 1 tau, 6 ratios, 9 weights, 8 normalisation) = 666, plus 9 flux
# products, 24 for three flux divergences, 18 Coriolis, 9 pressure and its
# gradients, 21 transports and vertical transport, 14 reference-profile terms,
# 12 AB2, 2 for the predicted tracer of the pressure, 4 slow-forcing sums and
# 3 surface forcing = 782.
TEND_FLOPS_PER_CELL = 782
# Barotropic stage (FP64), per column and launch of up to 7 substeps: read
# eta, U, V, G_U, G_V and the wet-layer count (half a word), the two transport
# sums (not in the first launch) and the three window sums (only once the
# averaging window has begun); write eta, U, V, the two transport sums and the
# three window sums (only once the window has begun), or in the last launch
# eta, U, V and the three step means; plus the copy back of eta, U, V after an
# odd number of launches. Summed over the launches of a step by
# baro_words_per_step().
BARO_FUSE = 7
# Column solve with the constant diffusivity: read u*, v*, T* and write u, v, T.
COLUMN_WORDS_PER_CELL = 6
# With salinity the tendency kernel also reads S', G_S^{n-1} and writes S'*,
# G_S^n (16 words per cell), and the column solve reads S'* and writes S' (8).
TEND_WORDS_PER_CELL_SALT = 16
COLUMN_WORDS_PER_CELL_SALT = 8
KERNEL_SOURCES = {"k_tend": "k_tend.hip", "k_baro_fused": "k_baro.hip", "k_column": "k_column.hip"}


def _src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _kernel_src(kernel):
    return os.path.join(ROOT, "paper_2309_06662_amd", "csrc", KERNEL_SOURCES[kernel])


def _traffic_from_profiles(workload, precision, kernel="k_tend"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_sha256_16") != _src_hash(_kernel_src(kernel)):
            return None
        return rec.get("hbm_bytes_per_launch")
    except Exception:
        return None


def run_gpu(w, precision, inp, steps, warmup):
    import torch

    from paper_2309_06662_amd import ocn

    m = ocn.Model(w, precision, inp)
    m.step(warmup)
    m.synchronize()
    m.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    m.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages, n = m.stage_times()
    m.stage_timing(False)
    diag = m.diagnostics(allow_unstable=True)
    m.close()
    del m
    torch.cuda.empty_cache()
    return elapsed, {k: v / max(n, 1) for k, v in stages.items()}, diag


def run_ensemble(steps, warmup, n_members=64):
    """64 seeded beta-plane basins of uneven sizes in FP32: batched stepping
    (one launch per stage, graph-replayed, autotuned tiles and schedule)
    against stepping each member alone with the same kernels, each member's
    step replayed from its own graph, and against the plain method (each
    member alone in FP64, graph-replayed); the two schedules of the batched
    launches (one workgroup per tile, persistent workgroups over per-XCD
    queues) at the default tiles; and the autotune cache: a second ensemble of
    the same shape takes the stored choice without timing."""
    import tempfile

    import torch

    from paper_2309_06662_amd import ocn

    ws = inputs.ensemble_members(n_members)
    ens = ocn.Ensemble(ws, "fp32")

    def timed(n):
        ens.step(warmup)
        ens.synchronize()
        t0 = time.perf_counter()
        ens.step(n)
        ens.synchronize()
        return time.perf_counter() - t0

    schedules = {}
    for name, pers in (("one_workgroup_per_tile", 0), ("persistent_queues", 1)):
        ens.set_tiles(0, 0, pers)
        schedules[name] = timed(steps) / steps * 1e3
    cache = os.path.join(tempfile.mkdtemp(prefix="ocn_autotune_"), "autotune.json")
    tune = ens.autotune(trial_steps=2, cache=cache)
    batched = timed(steps)
    # the same members one by one, each step replayed from its own captured
    # graph (two warm-up steps capture the graphs of both history buffers)
    seq = lambda: [ocn._check(ocn.lib().ocn_step_graph(mem.handle, 1), "ocn_step_graph") for mem in ens.members]
    for _ in range(2):
        seq()
    ens.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq()
    ens.synchronize()
    sequential = time.perf_counter() - t0
    diags = [m.diagnostics(allow_unstable=True) for m in ens.members]
    finite = all(d["nonfinite"] == 0 for d in diags)
    cells = ens.cells
    ens.close()
    del ens
    torch.cuda.empty_cache()
    # the plain method: each member alone in FP64, its step replayed from its own graph
    side = torch.cuda.Stream()
    plain = [ocn.Model(w, "fp64", inputs.make_inputs(w), stream=side) for w in ws]
    for _ in range(2):
        for mem in plain:
            mem.step(1, graph=True)
    side.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for mem in plain:
            mem.step(1, graph=True)
    side.synchronize()
    plain64 = time.perf_counter() - t0
    finite = finite and all(mem.diagnostics(allow_unstable=True)["nonfinite"] == 0 for mem in plain)
    for mem in plain:
        mem.close()
    del plain
    torch.cuda.empty_cache()
    ens2 = ocn.Ensemble(ws, "fp32")
    t0 = time.perf_counter()
    again = ens2.autotune(trial_steps=2, cache=cache)
    again = dict(again, seconds=round(time.perf_counter() - t0, 3))
    ens2.close()
    del ens2
    torch.cuda.empty_cache()
    return {"members": n_members, "cells": cells, "precision": "fp32", "steps": steps,
            "batched_ms_per_step": batched / steps * 1e3,
            "batched_cell_updates_per_s": cells * steps / batched,
            "sequential_ms_per_step": sequential / steps * 1e3,
            "sequential_cell_updates_per_s": cells * steps / sequential,
            "speedup_batched_over_sequential": sequential / batched,
            "sequential_mode": "each member replayed from its own captured graph",
            "plain_fp64_sequential_ms_per_step": plain64 / steps * 1e3,
            "speedup_batched_fp32_over_plain_fp64": plain64 / batched,
            "schedules_ms_per_step_default_tiles": schedules,
            "autotune": tune, "autotune_cache_second_ensemble": again,
            "finite": finite, "max_abs_u": max(d["max_abs_u"] for d in diags)}


def run_small(steps=200, warmup=5):
    """The 64 x 64 x 16 beta-plane basin: cache-resident and bound by launch
    latency, so it reports microseconds per step stepped eagerly and replayed
    from a captured graph."""
    import torch

    from paper_2309_06662_amd import ocn

    w = inputs.BETA_BASIN_64
    inp = inputs.make_inputs(w)
    out = {"workload": w.name}
    for prec in ("fp64", "fp32"):
        side = torch.cuda.Stream()
        m = ocn.Model(w, prec, inp, stream=side)
        rec = {}
        for mode in ("eager", "graph"):
            m.step(warmup, graph=(mode == "graph"))
            m.synchronize()
            t0 = time.perf_counter()
            m.step(steps, graph=(mode == "graph"))
            m.synchronize()
            rec[f"{mode}_us_per_step"] = (time.perf_counter() - t0) / steps * 1e6
        rec["graph_speedup"] = rec["eager_us_per_step"] / rec["graph_us_per_step"]
        out[prec] = rec
        m.close()
    return out


def run_salinity(w, steps, warmup):
    """The same workload with salinity and the quadratic equation of state
    (FP32): time per step, stages and the roofline of the salinity variant of
    the tendency kernel (16 words per cell) and of the column solve (8)."""
    import torch

    ws = w.replace(salinity=True)
    inp = inputs.make_inputs(ws)
    el, stages, diag = run_gpu(ws, "fp32", inp, steps, warmup)
    del inp
    ms = el / steps * 1e3
    cells = ws.cells
    tb = TEND_WORDS_PER_CELL_SALT * 4 * cells
    cb = COLUMN_WORDS_PER_CELL_SALT * 4 * cells
    t_s, c_s = stages["tendency"] * 1e-3, stages["column"] * 1e-3
    torch.cuda.empty_cache()
    return {"workload": ws.name + "_salinity", "ms_per_step": ms,
            "cell_updates_per_s": metrics.cell_updates_per_second(ws.nx, ws.ny, ws.nz, steps, el),
            "sypd": metrics.sypd(ws.dt, ms * 1e-3), "stage_ms": {k: round(v, 4) for k, v in stages.items()},
            "finite": diag["nonfinite"] == 0, "max_abs_u": diag["max_abs_u"],
            "tend_roofline": {"bound": "hbm", "bytes_per_launch": tb, "achieved": round(tb / t_s / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(tb / t_s / 1e9 / HBM_PEAK_GBS, 4)},
            "column_roofline": {"bound": "hbm", "bytes_per_launch": cb, "achieved": round(cb / c_s / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(cb / c_s / 1e9 / HBM_PEAK_GBS, 4)}}


def run_vector_invariant(w, steps, warmup):
    """The same workload with vector-invariant momentum advection (FP32): time
    per step, stages and the tendency kernel's roofline (the same 12 words per
    cell as the flux form: only the arithmetic between them differs)."""
    import torch

    wv = w.replace(momentum_form="vector_invariant")
    inp = inputs.make_inputs(wv)
    el, stages, diag = run_gpu(wv, "fp32", inp, steps, warmup)
    del inp
    ms = el / steps * 1e3
    tb = TEND_WORDS_PER_CELL * 4 * wv.cells
    t_s = stages["tendency"] * 1e-3
    torch.cuda.empty_cache()
    return {"workload": wv.name + "_vector_invariant", "ms_per_step": ms,
            "cell_updates_per_s": metrics.cell_updates_per_second(wv.nx, wv.ny, wv.nz, steps, el),
            "sypd": metrics.sypd(wv.dt, ms * 1e-3), "stage_ms": {k: round(v, 4) for k, v in stages.items()},
            "finite": diag["nonfinite"] == 0, "max_abs_u": diag["max_abs_u"],
            "tend_roofline": {"bound": "hbm", "bytes_per_launch": tb, "achieved": round(tb / t_s / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(tb / t_s / 1e9 / HBM_PEAK_GBS, 4)}}


def run_quarter(steps, warmup):
    """The 1/4-degree basin (1440 x 600 x 50) in both precisions, and the
    learned closure's cost there: the same FP32 step with a 208-128-128-50
    network (random weights) evaluated for every column at every step."""
    import torch

    from paper_2309_06662_amd import ocn

    w = inputs.LATLON_QUARTER
    inp = inputs.make_inputs(w)
    out = {"workload": w.name}
    for prec in ("fp32", "fp64"):
        el, stages, diag = run_gpu(w, prec, inp, steps, warmup)
        ms = el / steps * 1e3
        out[prec] = {"ms_per_step": ms, "cell_updates_per_s": w.cells * steps / el,
                     "sypd": metrics.sypd(w.dt, ms * 1e-3), "stage_ms": {k: round(v, 4) for k, v in stages.items()},
                     "finite": diag["nonfinite"] == 0, "max_abs_u": diag["max_abs_u"]}
    din, h, dout = (4 * w.nz + 3 + 7) // 8 * 8, 128, w.nz
    rng = np.random.default_rng(0)
    P = [rng.normal(size=(din, h)) * np.sqrt(2.0 / din), np.zeros(h), rng.normal(size=(h, h)) * np.sqrt(2.0 / h),
         np.zeros(h), rng.normal(size=(h, dout)) * 0.01, np.full(dout, -5.0)]
    net = ocn.Mlp(din, h, h, dout, max_batch=1024)
    net.set_params(np.concatenate([p.reshape(-1) for p in P]).astype(np.float32))
    norm = np.concatenate([np.zeros(din), np.ones(din)]).astype(np.float32)
    m = ocn.Model(w, "fp32", inp)
    m.attach_closure(net, norm)
    m.step(warmup)
    m.synchronize()
    m.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    m.synchronize()
    el = time.perf_counter() - t0
    st, n = m.stage_times()
    m.stage_timing(False)
    dg = m.diagnostics(allow_unstable=True)
    m.detach_closure()
    m.close()
    cols = w.nx * w.ny
    gemm_flops = 2.0 * cols * (din * h + h * h + h * dout)
    cl_ms = st["closure"] / max(n, 1)
    out["closure"] = {"network": [din, h, h, dout], "ms_per_step": el / steps * 1e3,
                      "closure_stage_ms": cl_ms, "slowdown_vs_constant_kappa": (el / steps * 1e3) / out["fp32"]["ms_per_step"],
                      "speedup_over_plain_fp64": out["fp64"]["ms_per_step"] / (el / steps * 1e3),
                      "network_tflops_in_closure_stage": gemm_flops / (cl_ms * 1e-3) / 1e12,
                      "finite": dg["nonfinite"] == 0, "max_abs_u": dg["max_abs_u"]}
    # Richardson-number mixing: viscosity and diffusivity diagnosed from the state every step
    m = ocn.Model(w, "fp32", inp)
    m.attach_closure()
    m.set_richardson()
    m.step(warmup)
    m.synchronize()
    m.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    m.synchronize()
    el = time.perf_counter() - t0
    st, n = m.stage_times()
    m.stage_timing(False)
    dg = m.diagnostics(allow_unstable=True)
    m.detach_closure()
    m.close()
    ri_ms = st["closure"] / max(n, 1)
    # the diagnosis reads T, u, v and writes the two face fields: 5 FP32 words per cell
    out["richardson"] = {"ms_per_step": el / steps * 1e3, "diagnosis_ms": ri_ms,
                         "diagnosis_gbs": 5 * 4 * w.cells / (ri_ms * 1e-3) / 1e9,
                         "column_ms": st["column"] / max(n, 1),
                         "slowdown_vs_constant_kappa": (el / steps * 1e3) / out["fp32"]["ms_per_step"],
                         "finite": dg["nonfinite"] == 0, "max_abs_u": dg["max_abs_u"]}
    return out


def copy_bandwidth(mib=2048, repeat=5):
    """Device-to-device copy bandwidth (read + write bytes / time) measured now."""
    import torch

    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeat):
        y.copy_(x)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * 4 * n * repeat / el / 1e9


def baro_words_per_step(n_substeps, fuse=BARO_FUSE):
    """FP64 words per column that the barotropic stage of one step must move."""
    M = n_substeps + n_substeps // 2
    qf = next((q for q in range(1, M + 1) if abs(q / n_substeps - 1.0) < 0.5), M + 1)
    words, launches = 0.0, 0
    for m0 in range(0, M, fuse):
        ss = min(fuse, M - m0)
        first, last = m0 == 0, m0 + ss == M
        rd = 5.5 + (0 if first else 2) + (3 if m0 >= qf else 0)
        wr = 6 if last else 3 + 2 + (3 if m0 + ss >= qf else 0)
        words += rd + wr
        launches += 1
    if launches % 2:
        words += 6
    return words, launches


def roofline(w, precision, stage_ms, n_baro_launches):
    """Rooflines of the three stages from their HIP-event times per step.

    Tendency: 12 words per cell, or 782 flops per cell against the vector
    peak, whichever fraction is larger (the dominant kernel). Barotropic: the
    FP64 words per column of baro_words_per_step(). Column solve: 6 words per
    cell."""
    esize = 4 if precision == "fp32" else 8
    t = stage_ms["tendency"] * 1e-3
    cells = w.cells
    gbs = TEND_WORDS_PER_CELL * esize * cells / t / 1e9
    tfl = TEND_FLOPS_PER_CELL * cells / t / 1e12
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    alu = {"bound": "alu", "achieved": round(tfl, 2), "peak": ALU_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
           "frac": round(tfl / ALU_PEAK_TFLOPS[precision], 4)}
    main, other = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    main = dict(main, kernel="k_tend", traffic=_traffic_from_profiles(w.name, precision, "k_tend"))
    cols = w.nx * w.ny
    words, _ = baro_words_per_step(w.n_substeps)
    baro_step_bytes = words * 8 * cols
    tb = stage_ms["barotropic"] * 1e-3
    baro = {"kernel": "k_baro_fused", "bound": "hbm", "launches_per_step": n_baro_launches,
            "words_per_column_step": words, "bytes_per_step": baro_step_bytes,
            "bytes_per_launch": round(baro_step_bytes / max(n_baro_launches, 1)),
            "achieved": round(baro_step_bytes / tb / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(baro_step_bytes / tb / 1e9 / HBM_PEAK_GBS, 4),
            "share_of_step": round(stage_ms["barotropic"] / sum(stage_ms[k] for k in ("tendency", "barotropic", "column")), 4),
            "traffic": _traffic_from_profiles(w.name, precision, "k_baro_fused")}
    col_bytes = COLUMN_WORDS_PER_CELL * esize * cells
    tc = stage_ms["column"] * 1e-3
    col = {"kernel": "k_column", "bound": "hbm", "bytes_per_launch": col_bytes,
           "achieved": round(col_bytes / tc / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(col_bytes / tc / 1e9 / HBM_PEAK_GBS, 4)}
    return main, other, {"barotropic": baro, "column": col}


# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per
# second (a wave64 instruction holds a SIMD for 4 cycles)
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9


def _valu_per_cell_from_profiles(workload, precision, path=None):
    """VALU lane-instructions per cell of the tendency kernel from the
    committed SQ counter summary, if it was taken on the current source."""
    path = path or os.path.join(ROOT, "profiles", f"sq_counters_{workload}_{precision}.txt")
    try:
        text = open(path).read()
    except OSError:
        return None
    want = f"# source sha256/16 of {KERNEL_SOURCES['k_tend']}: {_src_hash(_kernel_src('k_tend'))}"
    if want not in text:
        return None
    block = text.split("ocn::k_tend<", 1)
    if len(block) < 2:
        return None
    for line in block[1].split("\n"):
        if "VALU lane-instructions per cell:" in line:
            return float(line.split("VALU lane-instructions per cell:")[1].split(";")[0])
    return None


def valu_issue_view(w, precision, stage_ms, per_cell=None):
    """The tendency kernel against the VALU issue rate: instructions per cell
    (SQ counters of the committed summary) x cells / the measured kernel time."""
    n = _valu_per_cell_from_profiles(w.name, precision) if per_cell is None else per_cell
    if n is None:
        return None
    rate = n * w.cells / (stage_ms["tendency"] * 1e-3)
    return {"kernel": "k_tend", "bound": "valu_issue", "instructions_per_cell": n,
            "achieved": round(rate / 1e12, 2), "peak": round(VALU_ISSUE_PEAK / 1e12, 2),
            "unit": "T lane-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4),
            "source": f"profiles/sq_counters_{w.name}_{precision}.txt"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_window_rate(args):
    """Steps one oracle window for about seconds; returns (cells x steps, seconds)."""
    import oracle

    w, lon0, seconds = args
    win = w.replace(name=w.name + "_window", nx=240, ny=120, periodic_x=False, x0=lon0, y0=-10.0)
    m = oracle.OracleModel.from_inputs(win, inputs.make_inputs(win))
    steps = 0
    t0 = time.perf_counter()
    while True:
        m.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds or steps >= 20:
            break
    m.close()
    return win.cells * steps, el, steps


def oracle_rates(w, seconds=10.0):
    """The oracle's rate on bounded windows of a workload: one 240 x 120
    column window (all levels) stepped for about `seconds` on one thread, then
    one such window per host core (at most 16, the host share of one GPU),
    each on its own thread (the oracle is serial; ctypes releases the
    interpreter lock)."""
    import concurrent.futures as cf

    cu1, el1, st1 = _oracle_window_rate((w, 150.0, seconds))
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    cores = max(1, min(16, ncpu))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(_oracle_window_rate, [(w, 10.0 + 20.0 * q, seconds) for q in range(cores)]))
    wall = time.perf_counter() - t0
    return {"one": cu1 / el1, "one_steps": st1, "one_s": el1, "all": sum(r[0] for r in res) / wall,
            "cores": cores, "all_steps": (min(r[2] for r in res), max(r[2] for r in res)), "all_s": wall,
            "host_cpus": ncpu}


def cpu_baseline(w):
    """The oracle as it stands (plain FP64 C, gcc -O2 -ffp-contract=off, the
    build the tests use) on bounded windows of the same 1/12-degree workload,
    one thread and all host cores (oracle_rates); beside it the same sources
    built -O3 -march=x86-64-v3 (no contraction: the same arithmetic), timed in
    a child process. The full grid is not run on the CPU."""
    import subprocess

    r = oracle_rates(w)
    o3 = None
    try:
        env = dict(os.environ, OCN_ORACLE_BUILD="o3")
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-rates", "--workload", w.name],
                             env=env, capture_output=True, text=True, timeout=300, check=True)
        o3 = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as exc:  # the -O3 figure is context only
        print(f"[bench] -O3 oracle timing skipped: {exc}", file=sys.stderr, flush=True)
    rec = {"value": r["one"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"240x120x100 window of the 1/12-degree basin (150-170E, 10S-0), {r['one_steps']} steps in "
                     f"{r['one_s']:.1f} s, FP64, one thread, gcc -O2 -ffp-contract=off",
           "all_cores": {"value": r["all"], "unit": "cell-updates/s", "cores": r["cores"],
                         "sample": f"{r['cores']} windows of 240x120x100 (10S-0, 20 degrees apart), one per thread, "
                                   f"{r['all_steps'][0]}-{r['all_steps'][1]} steps each in {r['all_s']:.1f} s"},
           "cpu_model": _cpu_model(), "host_cpus": r["host_cpus"]}
    if o3 is not None:
        rec["o3_build"] = {"flags": "gcc -O3 -march=x86-64-v3 -ffp-contract=off", "one_thread": o3["one"],
                           "all_cores": o3["all"], "cores": o3["cores"], "unit": "cell-updates/s"}
    return rec


def copy_probe(mib=1024, repeat=3):
    """A plain device-to-device copy of known size, for calibrating the
    memory-traffic counters: under a counter collector, the bytes the counters
    report for the copy kernel are compared with the bytes it must move."""
    import torch

    n = mib * (1 << 20) // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(repeat):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_floats": n, "bytes_read": 4 * n, "bytes_written": 4 * n, "repeat": repeat}))


def _per_dispatch(path, counter, name_part):
    """Counter values per dispatch of kernels whose name contains name_part, in dispatch order."""
    import csv

    vals = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter or name_part not in r.get("Kernel_Name", ""):
                continue
            d = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
            vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return [vals[d] for d in sorted(vals)]


def pmc_summary(a):
    """Per-launch HBM traffic of a kernel from the counter_collection.csv files
    of four rocprofv3 runs: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
    benchmark and of the copy probe. The copy reads and writes a known number
    of bytes; the ratio of those bytes to its counters scales the kernel's. The
    record keeps the hash of the kernel's source so that a reader can tell
    whether it still applies."""
    cf_ = _per_dispatch(a.copy_fetch, "FETCH_SIZE", "copy")
    cw_ = _per_dispatch(a.copy_write, "WRITE_SIZE", "copy")
    kf = _per_dispatch(a.fetch, "FETCH_SIZE", a.name or a.kernel)
    kw = _per_dispatch(a.write, "WRITE_SIZE", a.name or a.kernel)
    if not (cf_ and cw_ and kf and kw):
        raise SystemExit("missing dispatches in the counter files")
    # the largest copy dispatch is the probe's copy; the last kernel dispatches are steady steps
    f_scale = a.copy_bytes / (max(cf_) * 1024.0)
    w_scale = a.copy_bytes / (max(cw_) * 1024.0)
    tail = kf[-a.steady:], kw[-a.steady:]
    fetch_b = sum(tail[0]) / len(tail[0]) * 1024.0 * f_scale
    write_b = sum(tail[1]) / len(tail[1]) * 1024.0 * w_scale
    rec = {"kernel": a.kernel, "dispatch_name_filter": a.name or a.kernel, "workload": a.workload,
           "precision": a.precision,
           "source_sha256_16": _src_hash(_kernel_src(a.kernel)),
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "steady_dispatches_averaged": a.steady,
           "copy_fetch_kib": max(cf_), "copy_write_kib": max(cw_), "copy_bytes": a.copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_fetch_bytes_per_launch": fetch_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": fetch_b + write_b, "commands": a.command}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("fetch_scale", "write_scale", "hbm_bytes_per_launch")}))


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_INSTS_SALU", "SQ_WAIT_INST_ANY",
               "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_WAVE_CYCLES",
               "SQ_THREAD_CYCLES_VALU", "GRBM_GUI_ACTIVE")


def sq_summary(a):
    """Text summary of two rocprofv3 SQ counter passes (counter_collection.csv
    of each) for the last dispatch of the tendency, barotropic and column
    kernels: the counters, VALU and LDS instructions per cell (per
    column-substep for the barotropic kernel) and VALU busy, taken as
    SQ_INSTS_VALU x 4 cycles (a wave64 VALU instruction holds a 16-lane SIMD
    for 4 cycles) over 1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs."""
    import csv

    def load(path):
        per = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                per.setdefault(key, {})
                per[key][r["Counter_Name"]] = per[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        return per

    w = inputs.WORKLOADS[a.workload]
    cells, cols = w.nx * w.ny * w.nz, w.nx * w.ny
    p1, p2 = load(a.sq1), load(a.sq2)
    # a run of both precisions steps FP32 first: the FP64 dispatches start at
    # the first FP64 tendency launch
    for p in (p1, p2):
        split = min([k[0] for k in p if "ocn::k_tend<double" in k[1]] or [1 << 62])
        for k in list(p):
            if (k[0] >= split) != (a.precision == "fp64"):
                del p[k]
    lines = [f"# rocprofv3 SQ counters of the last dispatch of each kernel, {a.precision.upper()} step of {w.name}"]
    lines += [f"# command: {c}" for c in a.command]
    lines += [f"# source sha256/16 of {KERNEL_SOURCES[k]}: {_src_hash(_kernel_src(k))}" for k in sorted(KERNEL_SOURCES)]
    lines += ["# VALU busy = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs); per-cell figures",
              "# are instructions x 64 lanes / cells (columns x substeps for the barotropic kernel)", ""]
    for part in ("ocn::k_tend<", "ocn::k_baro_fused<", "ocn::k_column<"):
        sel = lambda p: sorted(k for k in p if part in k[1])
        if part == "ocn::k_baro_fused<":  # the launches of the full substep count, not a step's shorter last one
            depth = lambda k: int(k[1].split("<")[1].split(">")[0].split(",")[2])
            sel = lambda p, _s=sel: [k for k in _s(p) if depth(k) == max(map(depth, _s(p)))]
        k1, k2 = sel(p1), sel(p2)
        if not (k1 and k2):
            continue
        c = dict(p1[k1[-1]])
        c.update(p2[k2[-1]])
        name = k1[-1][1].split("(")[0]
        if part == "ocn::k_baro_fused<":
            sh = int(name.split("<")[1].split(">")[0].split(",")[2])
            n, unit = cols * sh, "column-substep"
        else:
            n, unit = cells, "cell"
        cyc = c["GRBM_GUI_ACTIVE"] / 8
        lines.append(f"{name} (dispatch {k1[-1][0]}/{k2[-1][0]}): {cyc:.0f} cycles per XCD "
                     f"({cyc / 2.4e9 * 1e3:.2f} ms at 2.4 GHz)")
        lines += [f"  {k:24s} {c[k]:.4e}" for k in SQ_COUNTERS if k in c]
        lines.append(f"  VALU lane-instructions per {unit}: {c['SQ_INSTS_VALU'] * 64 / n:.0f}; LDS per {unit}: "
                     f"{c['SQ_INSTS_LDS'] * 64 / n:.1f}; SALU/VALU {c['SQ_INSTS_SALU'] / c['SQ_INSTS_VALU']:.2f}")
        lines.append(f"  VALU busy {c['SQ_INSTS_VALU'] * 4 / (1024 * cyc):.2f}; LDS bank-conflict cycles / LDS active "
                     f"cycles {c['SQ_LDS_BANK_CONFLICT'] / max(c['SQ_LDS_IDX_ACTIVE'], 1):.3f}; waves {c['SQ_WAVES']:.0f}")
        lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def stats_summary(a):
    """Text summary of a rocprofv3 --kernel-trace --stats run: the per-kernel
    table (microseconds) and, for a tendency kernel launched at most 24
    times (one workload), the duration of every launch with the mean of the
    steady ones (the first launch of a run is the forward-Euler start step)."""
    import csv

    rows = list(csv.DictReader(open(os.path.join(a.stats_dir, "run_kernel_stats.csv"))))
    lines = [f"# rocprofv3 kernel summary of {a.workload} (durations in microseconds)"]
    lines += [f"# command: {c}" for c in a.command]
    lines.append(f"{'kernel':72s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
    for r in rows:
        name = r["Name"][:72]
        lines.append(f"{name:72s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e3:12.1f} "
                     f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['MinNs']) / 1e3:10.1f} "
                     f"{float(r['MaxNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")
    per = {}
    for r in csv.DictReader(open(os.path.join(a.stats_dir, "run_kernel_trace.csv"))):
        if "ocn::k_tend<" in r["Kernel_Name"]:
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            per.setdefault(name, []).append((int(r["Dispatch_Id"]),
                                             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    for name, calls in per.items():
        if len(calls) > 24:  # launches of several workloads: the table's figures stand alone
            continue
        us = [d for _, d in sorted(calls)]
        steady = us[1:] or us
        lines.append(f"# {name} per call: {', '.join(f'{d:.1f}' for d in us)}; steady (AB2) mean "
                     f"{sum(steady) / len(steady):.1f} us")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=inputs.LATLON_TWELFTH.name, choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble measurement")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the small-basin graph timing, the 1/4-degree runs and the copy bandwidth")
    ap.add_argument("--no-salinity", action="store_true", help="skip the salinity leg")
    ap.add_argument("--no-vi", action="store_true", help="skip the vector-invariant momentum leg")
    ap.add_argument("--oracle-rates", action="store_true",
                    help="print the oracle's one-thread and all-cores rates as JSON and exit (no GPU)")
    ap.add_argument("--copy-probe", action="store_true", help="run the counter-calibration copy and exit")
    ap.add_argument("--mib", type=int, default=1024, help="copy probe: size of each buffer in MiB")
    ap.add_argument("--pmc-summary", action="store_true", help="write a kernel's traffic record and exit")
    ap.add_argument("--sq-summary", action="store_true", help="write the SQ counter summary of two passes and exit")
    ap.add_argument("--stats-summary", action="store_true", help="write the kernel summary of a --stats run and exit")
    ap.add_argument("--stats-dir", help="stats summary: the rocprofv3 output directory")
    ap.add_argument("--sq1", help="sq summary: counter_collection.csv of the first pass")
    ap.add_argument("--sq2", help="sq summary: counter_collection.csv of the second pass")
    ap.add_argument("--kernel", default="k_tend", choices=sorted(KERNEL_SOURCES))
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, help="bytes the copy kernel reads (= writes)")
    ap.add_argument("--steady", type=int, default=1, help="pmc summary: average of the last N dispatches")
    ap.add_argument("--name", help="pmc summary: substring of the dispatches' kernel name (default: --kernel)")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out")
    args = ap.parse_args()

    if args.copy_probe:
        copy_probe(args.mib)
        return
    if args.oracle_rates:
        print(json.dumps(oracle_rates(inputs.WORKLOADS[args.workload])))
        return
    if args.pmc_summary:
        pmc_summary(argparse.Namespace(**{**vars(args), "workload": args.workload}))
        return
    if args.sq_summary:
        sq_summary(args)
        return
    if args.stats_summary:
        stats_summary(args)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    w = inputs.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    inp = inputs.make_inputs(w)
    print(f"[bench] inputs for {w.name} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    results = {}
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp64"]):
        el, stages, diag = run_gpu(w, prec, inp, args.steps, args.warmup)
        ms = el / args.steps * 1e3
        results[prec] = {
            "ms_per_step": ms,
            "cell_updates_per_s": metrics.cell_updates_per_second(w.nx, w.ny, w.nz, args.steps, el),
            "sypd": metrics.sypd(w.dt, ms * 1e-3),
            "stage_ms": {k: round(v, 4) for k, v in stages.items()},
            "finite": diag["nonfinite"] == 0,
            "max_abs_u": diag["max_abs_u"],
            "steps_taken": args.warmup + args.steps,
        }
        print(f"[bench] {prec}: {ms:.3f} ms/step, stages {results[prec]['stage_ms']}, "
              f"finite={diag['nonfinite'] == 0}", file=sys.stderr, flush=True)

    sal = None
    if not args.no_salinity:
        sal = run_salinity(w, args.steps, args.warmup)
        print(f"[bench] salinity fp32: {sal['ms_per_step']:.3f} ms/step, stages {sal['stage_ms']}, "
              f"finite={sal['finite']}", file=sys.stderr, flush=True)

    vi = None
    if not args.no_vi:
        vi = run_vector_invariant(w, args.steps, args.warmup)
        print(f"[bench] vector-invariant fp32: {vi['ms_per_step']:.3f} ms/step, stages {vi['stage_ms']}, "
              f"finite={vi['finite']}", file=sys.stderr, flush=True)

    ens = None
    if not args.no_ensemble:
        ens = run_ensemble(args.steps, args.warmup)
        print(f"[bench] ensemble: batched {ens['batched_ms_per_step']:.3f} ms/step, sequential "
              f"{ens['sequential_ms_per_step']:.3f} ms/step, plain FP64 one by one "
              f"{ens['plain_fp64_sequential_ms_per_step']:.3f} ms/step, tiles {ens['autotune']}",
              file=sys.stderr, flush=True)

    extra = {}
    if not args.no_extra:
        extra["copy_gbs"] = copy_bandwidth()
        extra["small"] = run_small()
        print(f"[bench] small basin: {extra['small']}", file=sys.stderr, flush=True)
        extra["quarter"] = run_quarter(args.steps, args.warmup)
        print(f"[bench] 1/4 degree: {extra['quarter']}", file=sys.stderr, flush=True)

    main_rec = results["fp32"]
    n_baro = baro_words_per_step(w.n_substeps)[1]  # launches per step
    roof, other, stage_roofs = roofline(w, "fp32", main_rec["stage_ms"], n_baro)
    if "copy_gbs" in extra and roof["unit"] == "GB/s":
        roof["frac_of_measured_copy"] = round(roof["achieved"] / extra["copy_gbs"], 4)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} cell-updates/s ({cpu['sample']})", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": main_rec["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic seeded basin (analytic seamount-and-ridge bathymetry, exponential stratification "
                "with N(0, 0.01) noise, cos-latitude wind, restoring)",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "dt_s": w.dt, "n_substeps": w.n_substeps,
                   "halo": w.halo, "precision": "FP32 bulk, FP64 barotropic substeps, averages and sums"},
        "sypd": main_rec["sypd"],
        "finite": main_rec["finite"],
        "max_abs_u": main_rec["max_abs_u"],
        "steps_taken": main_rec["steps_taken"],
        "stage_ms": main_rec["stage_ms"],
        "roofline": roof,
        "roofline_other_view": other,
        "roofline_valu_issue": valu_issue_view(w, "fp32", main_rec["stage_ms"]),
        "stage_rooflines": stage_roofs,
        "cpu_baseline": cpu,
    }
    if "fp64" in results:
        r64 = results["fp64"]
        r64_main, _, r64_stages = roofline(w, "fp64", r64["stage_ms"], n_baro)
        line["fp64"] = {"value": r64["cell_updates_per_s"], "ms_per_step": r64["ms_per_step"], "sypd": r64["sypd"],
                        "finite": r64["finite"], "max_abs_u": r64["max_abs_u"],
                        "stage_ms": r64["stage_ms"], "roofline": r64_main, "stage_rooflines": r64_stages}
        line["fp32_speedup_over_fp64"] = r64["ms_per_step"] / main_rec["ms_per_step"]
    if sal is not None:
        line["salinity"] = sal
    if vi is not None:
        line["vector_invariant"] = vi
    if ens is not None:
        line["ensemble"] = ens
    line.update(extra)
    print(json.dumps(line), flush=True)
    if not main_rec["finite"]:
        print("[bench] the headline leg ended with non-finite values: its throughput is not a valid measurement",
              file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()
