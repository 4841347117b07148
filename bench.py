"""Benchmark: emissivity solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2_batched]
                    [--no-cpu-baseline]

A step is one solve of the whole batched workload (16384 cells x 32
carbonaceous radii, 500 wavelengths; 524,288 (cell, grain) pairs): the fused
rates/recursion kernels, the emission contraction and the energy diagnostics,
replayed from a plan (HIP graphs captured once, solver classes as parallel
branches) with the solver's launch configuration chosen by the autotuner
(cached in paper_1311_4627_amd/tuned.json; timing it again takes seconds and
is not part of the timed region).  Fields are resident in HBM before the
timed region; j_lambda and the diagnostics stay on the device.  Prints one
JSON line.

The roofline object covers the dominant phase (the fused rates/recursion
kernels), timed with HIP events on the solve's stream inside the timed steps.
Its bound is the transcendental pipe: every upward rate needs one v_exp_f32,
which issues at a quarter of the FP32 FMA rate (157.3 TFLOP/s = 78.6e12 FMA/s),
so the chip evaluates at most 19.66e12 rates/s.  The HBM traffic of that phase
comes from the rocprofv3 FETCH_SIZE/WRITE_SIZE summary committed under
profiles/, and is reported only while the solver sources still hash to the
values recorded there.

The CPU baseline is the FP64 oracle timed on the host cores over a bounded,
stratified sample of the same workload (a few cells times every radius); the
one-time per-grain setup is excluded, as the GPU's per-grain precompute is.
It runs before anything touches the GPU.  The oracle's spectra of that sample
are then compared with the timed run's own output for the same pairs
(oracle_error: the largest relative error on j_lambda over the wavelengths
within 1e-10 of each spectrum's maximum, against the 1e-4 bar).
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from synth.fields import make_fields  # noqa: E402

METRIC = "emissivity solves/s (cell×grain) at 1e-4 rel err; surrogate vs plain speedup"
J_TOL = 1e-4                                 # end-to-end bar on j_lambda against the oracle
EXP2_PEAK = 157.3e12 / 2 / 4                 # v_exp_f32 per second: a quarter of the FP32 FMA rate
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve_c2_hbm_traffic.md")
TUNE_CACHE = os.path.join(ROOT, "paper_1311_4627_amd", "tuned.json")
# the solver kernel's own sources (the traffic summary is valid while they are unchanged)
SOLVER_SOURCES = ["paper_1311_4627_amd/csrc/hsd_solve.hip", "paper_1311_4627_amd/csrc/hsd_index.h"]


def solver_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SOLVER_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per solve phase from the committed counter summary, or None
    when the summary is missing or was taken on other solver sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("solver_sources_sha256_16:"):
            vals["hash"] = line.split(":", 1)[1].strip()
        if line.startswith("solve_phase_hbm_bytes_per_step:"):
            vals["bytes"] = float(line.split(":", 1)[1].strip())
    if vals.get("hash") != solver_hash() or "bytes" not in vals:
        return None
    return vals["bytes"]


def _oracle_task(args):
    name, gi, cells = args
    import oracle
    w = synth.workload(name)
    g = w.grains[gi]
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells, cells=np.asarray(cells))
    oracle.grain_setup(g, w.lam_cm)                       # one-time setup, not timed
    t0 = time.perf_counter()
    js = [oracle.solve_pair(u[c], g, w.lam_cm)[1] for c in range(len(cells))]
    return time.perf_counter() - t0, len(cells), gi, list(cells), np.stack(js)


def cpu_baseline(name: str, cells_per_grain: int):
    """The oracle timed over a seeded sample of the workload's pairs; returns
    the baseline record and the oracle's spectra of the sample as
    (grain index, cells, j [cells][L]) triples."""
    w = synth.workload(name)
    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(4627)
    tasks = []
    for gi in range(len(w.grains)):
        cells = sorted(rng.choice(w.n_cells, size=cells_per_grain, replace=False).tolist())
        tasks.append((name, gi, cells))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_task, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    busy = sum(r[0] for r in res)
    pairs = sum(r[1] for r in res)
    # pairs per second of solve work on `cores` cores (setup excluded)
    rate = pairs / busy * cores
    rec = {"value": rate, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"{cells_per_grain} seeded cells x {len(w.grains)} radii of {name} "
                     f"({pairs} pairs, {busy:.1f} core-s of solve work, {wall:.1f} s wall incl. per-grain setup)"}
    return rec, [(r[2], r[3], r[4]) for r in res]


def j_rel_err(j: np.ndarray, jref: np.ndarray) -> float:
    """Largest |j / j_ref - 1| over the wavelengths where j_ref is at least
    1e-10 of the spectrum's maximum (the range the 1e-4 bar covers)."""
    if jref.max() <= 0.0:
        return 0.0 if np.all(j == 0.0) else math.inf
    m = jref >= 1e-10 * jref.max()
    return float(np.max(np.abs(j[m] / jref[m] - 1.0))) if np.any(m) else 0.0


def oracle_error(j, samples) -> dict:
    """Error of the timed run's last spectra against the oracle's, pair by pair."""
    import torch
    worst, n = 0.0, 0
    for gi, cells, jr in samples:
        idx = torch.tensor(cells, dtype=torch.long, device=j.device)
        got = j[:, gi].index_select(0, idx).cpu().numpy().astype(np.float64)
        for c in range(len(cells)):
            worst = max(worst, j_rel_err(got[c], jr[c]))
            n += 1
    return {"pairs": n, "max_rel_err_j": worst, "tol": J_TOL, "within_tol": bool(worst <= J_TOL)}


def count_rates(ctx_tables, lam, grain) -> int:
    """Algorithmic upward-rate evaluations of one pair: the transitions f > i
    whose photon wavelength hc / (E_f - E_i) lies on the wavelength grid."""
    E = ctx_tables[0]
    n = E.shape[0]
    hc = synth.CONSTANTS["h"] * synth.CONSTANTS["c"]
    emin, emax = hc / lam[-1], hc / lam[0]
    tot = 0
    for i in range(n - 1):
        d = E[i + 1:] - E[i]
        tot += int(np.count_nonzero((d >= emin) & (d <= emax)))
    return tot


def _band_error(jp, jr, lam):
    """Per pair: max over bands holding >= 1e-3 of the reference's emitted
    power of |J_b / J_b,ref - 1| (the bands and rule of the surrogate's
    accuracy metric; the same definition as the reference MLP's)."""
    L = lam.shape[0]
    e = (np.arange(33) * (L - 1)) // 32
    def bands(f):
        seg = 0.5 * (f[:, 1:] + f[:, :-1]) * np.diff(lam)
        cs = np.concatenate([np.zeros((f.shape[0], 1)), np.cumsum(seg, axis=1)], axis=1)
        return cs[:, e[1:]] - cs[:, e[:-1]]
    J, Jr = bands(jp.astype(np.float64)), bands(jr.astype(np.float64))
    m = Jr >= 1e-3 * Jr.sum(axis=1, keepdims=True)
    return np.where(m, np.abs(J / np.where(m, Jr, 1.0) - 1.0), 0.0).max(axis=1)


def radius_groups(grains, comp: str, n_groups: int):
    """The composition's grains split into n_groups ranges of consecutive
    radii (the workloads list radii in increasing order): (index, grain)
    lists, one network each."""
    sel = [(i, g) for i, g in enumerate(grains) if g.composition == comp]
    G = len(sel)
    return [sel[q * G // n_groups:(q + 1) * G // n_groups] for q in range(n_groups)]


def train_surrogates(torch, hsd, ctx, w4, ids, steps, batch, lr, log, n_groups=4):
    """Per composition and range of radii: plain-solve the training cells for
    those radii, build inputs and targets, fit the statistics and train one
    network; then the held-out band errors.  Returns the networks keyed by
    grain index and a report per composition."""
    from synth import surrogate as ssur
    nets, report = {}, {}
    u = torch.tensor(make_fields(w4.lam_cm, w4.field_recipe, w4.n_cells), device="cuda:0")
    nh = w4.notes["heldout_cells"]
    uh = torch.tensor(make_fields(w4.lam_cm, w4.notes["heldout_recipe"], nh), device="cuda:0")
    for comp in ("carbonaceous", "silicate"):
        errs, rerrs, terrs, groups = [], [], [], []
        n_tot, gen_tot, train_tot, loss_first, loss_last = 0, 0.0, 0.0, [], []
        for part in radius_groups(w4.grains, comp, n_groups):
            sel = [ids[i] for i, _ in part]
            G = len(sel)
            t0 = time.perf_counter()
            n = w4.n_cells * G
            j = torch.empty((w4.n_cells, G, w4.n_lambda), dtype=torch.float32, device="cuda:0")
            ctx.hsd_solve(u, sel, j, None)
            X = torch.empty((n, 33), dtype=torch.float32, device="cuda:0")
            A = torch.empty((n,), dtype=torch.float64, device="cuda:0")
            ctx.hsd_sur_features(u, sel, X, A)
            Y = torch.empty((n, ssur.n_outputs(w4.n_lambda)), dtype=torch.float32, device="cuda:0")
            ctx.hsd_sur_targets(j.view(n, w4.n_lambda), A, Y)
            ctx.hsd_sync()
            del j
            gen_s = time.perf_counter() - t0
            sur = hsd.Surrogate(ctx)
            sur.hsd_sur_set_params(ssur.init_params(ssur.n_outputs(w4.n_lambda)))
            sur.hsd_sur_fit_norm(X, Y)
            t0 = time.perf_counter()
            trace = sur.hsd_sur_train(X, Y, steps=steps, batch=batch, lr=lr)
            torch.cuda.synchronize()
            train_s = time.perf_counter() - t0
            # held-out cells: plain vs surrogate
            jr = torch.empty((nh, G, w4.n_lambda), dtype=torch.float32, device="cuda:0")
            jp = torch.empty_like(jr)
            dr = torch.empty((nh, G, 4), dtype=torch.float32, device="cuda:0")
            dp = torch.empty_like(dr)
            ctx.hsd_solve(uh, sel, jr, dr)
            sur.hsd_sur_predict(uh, sel, jp, dp)
            ctx.hsd_sync()
            err = _band_error(jp.cpu().numpy().reshape(-1, w4.n_lambda), jr.cpu().numpy().reshape(-1, w4.n_lambda),
                              w4.lam_cm)
            # the energy-ratio output against the plain model's emitted / absorbed
            drn = dr.cpu().numpy().reshape(-1, 4).astype(np.float64)
            dpn = dp.cpu().numpy().reshape(-1, 4).astype(np.float64)
            rerr = np.abs((dpn[:, 2] / dpn[:, 0]) / (drn[:, 1] / drn[:, 0]) - 1)
            # the cheap method the surrogate replaces: a table of training spectra
            # indexed by the field's total energy alone (nearest training cell, same
            # grain), scaled by the pair's own absorbed power
            Xh = torch.empty((nh * G, 33), dtype=torch.float32, device="cuda:0")
            Ah = torch.empty((nh * G,), dtype=torch.float64, device="cuda:0")
            ctx.hsd_sur_features(uh, sel, Xh, Ah)
            etot_t = torch.log10((10.0 ** X.view(w4.n_cells, G, 33)[:, 0, :32].double()).sum(dim=1))
            etot_h = torch.log10((10.0 ** Xh.view(nh, G, 33)[:, 0, :32].double()).sum(dim=1))
            nn = torch.argmin((etot_h[:, None] - etot_t[None, :]).abs(), dim=1)
            rows = (nn[:, None] * G + torch.arange(G, device="cuda:0")[None, :]).reshape(-1)
            jt = (10.0 ** Y.index_select(0, rows)[:, :w4.n_lambda].double()) * Ah[:, None]
            terr = _band_error(jt.cpu().numpy(), jr.cpu().numpy().reshape(-1, w4.n_lambda), w4.lam_cm)
            del X, Y, A, Xh, Ah, jt, jr, jp, dr, dp
            r0, r1 = part[0][1].radius_cm * 1e8, part[-1][1].radius_cm * 1e8
            groups.append({"radii_A": [round(r0, 1), round(r1, 1)], "train_pairs": n,
                           "heldout_band_err": {"median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                                                "max": float(err.max())}})
            log(f"{comp} {r0:.1f}-{r1:.1f} A: trained {steps} steps in {train_s:.1f} s; held-out band error median "
                f"{np.median(err):.4f} p99 {np.quantile(err, 0.99):.4f} max {err.max():.4f}")
            errs.append(err)
            rerrs.append(rerr)
            terrs.append(terr)
            n_tot += n
            gen_tot += gen_s
            train_tot += train_s
            loss_first.append(float(np.mean(trace[:20])))
            loss_last.append(float(np.mean(trace[-100:])))
            for i, _ in part:
                nets[i] = sur
        err, rerr, terr = np.concatenate(errs), np.concatenate(rerrs), np.concatenate(terrs)
        report[comp] = {"train_pairs": n_tot, "heldout_pairs": int(err.size), "networks": len(groups),
                        "steps": steps, "batch": batch, "data_s": round(gen_tot, 2), "train_s": round(train_tot, 2),
                        "loss_first": float(np.mean(loss_first)), "loss_last": float(np.mean(loss_last)),
                        "heldout_band_err": {"median": float(np.median(err)), "p90": float(np.quantile(err, 0.9)),
                                             "p99": float(np.quantile(err, 0.99)), "max": float(err.max())},
                        "heldout_energy_ratio_err": {"median": float(np.median(rerr)),
                                                     "p99": float(np.quantile(rerr, 0.99)), "max": float(rerr.max())},
                        "table_baseline_band_err": {"median": float(np.median(terr)),
                                                    "p99": float(np.quantile(terr, 0.99)),
                                                    "max": float(terr.max())},
                        "per_radius_range": groups}
        log(f"{comp}: {len(groups)} networks; held-out band error median {np.median(err):.4f} "
            f"p99 {np.quantile(err, 0.99):.4f} max {err.max():.4f}; "
            f"table method median {np.median(terr):.4f} p99 {np.quantile(terr, 0.99):.4f}")
    del u, uh
    return nets, report


def bench_surrogate(args):
    import torch
    from paper_1311_4627_amd import autotune, hsd

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    w4 = synth.workload("c4_train")
    ctx = hsd.Context(w4.lam_cm, device=0)
    ids = [ctx.add_grain(g) for g in w4.grains]
    nets, report = train_surrogates(torch, hsd, ctx, w4, ids, args.train_steps, 4096, 4e-3, log,
                                    args.radius_groups)
    if args.workload == "c4_train":
        tot_pairs = sum(r["train_pairs"] for r in report.values())
        tot_s = sum(r["train_s"] for r in report.values())
        n_nets = sum(r["networks"] for r in report.values())
        line = {"metric": "surrogate training: samples per second (held-out band errors reported)",
                "value": args.train_steps * 4096 * n_nets / tot_s, "unit": "samples/s", "n_gpus": 1,
                "steps": args.train_steps, "warmup": 0, "ms_per_step": 1e3 * tot_s / (args.train_steps * n_nets),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 matmul, f32 master",
                "data": "synthetic", "config": {"workload": "c4_train", "train_pairs": tot_pairs,
                                                "net": "33-256-256-256-501 GELU",
                                                "networks_per_composition": args.radius_groups},
                "per_composition": report}
        print(json.dumps(line))
        return
    # c5: 262144 cells x 64 radii x 2 compositions, plain vs surrogate + fallback
    w5 = synth.workload("c5_surrogate")
    assert [(g.composition, g.radius_cm) for g in w5.grains] == [(g.composition, g.radius_cm) for g in w4.grains]
    surs = [nets[gi] for gi in range(len(w5.grains))]
    u = torch.tensor(make_fields(w5.lam_cm, w5.field_recipe, w5.n_cells), device="cuda:0")
    G = len(ids)
    jpl = torch.empty((w5.n_cells, G, w5.n_lambda), dtype=torch.float32, device="cuda:0")
    dpl = torch.empty((w5.n_cells, G, 4), dtype=torch.float32, device="cuda:0")
    tuned = autotune.tune(ctx, u, ids, cache_path=TUNE_CACHE)
    log(f"c5 launch configuration: {tuned['cfg']} (cached: {tuned['cached']})")
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, out

    t_plain, _ = timed(lambda: ctx.hsd_solve(u, ids, jpl, dpl, stream), args.steps)
    log(f"plain: {t_plain * 1e3:.1f} ms per step")
    jsu = torch.empty_like(jpl)
    dsu = torch.empty_like(dpl)
    # the check against the absorbed power itself first (its results are not kept)
    t_abs, nfb_abs = timed(lambda: ctx.hsd_solve_surrogate(u, ids, surs, jsu, dsu, tol=0.01, check=hsd.CHECK_ABSORBED,
                                                           stream=stream), 1)
    log(f"surrogate + fallback, check against A: {t_abs * 1e3:.1f} ms, {nfb_abs} fallback pairs")
    n_pairs = w5.n_cells * G
    rng = np.random.default_rng(4627005)
    samp = np.sort(rng.choice(n_pairs, n_pairs // 100, replace=False))
    idx = torch.tensor(samp, device="cuda:0")
    jr = jpl.view(n_pairs, -1).index_select(0, idx).cpu().numpy()
    e_abs = _band_error(jsu.view(n_pairs, -1).index_select(0, idx).cpu().numpy(), jr, w5.lam_cm)
    t_sur, nfb = timed(lambda: ctx.hsd_solve_surrogate(u, ids, surs, jsu, dsu, tol=0.01, check=hsd.CHECK_MODEL,
                                                       stream=stream), args.steps)
    log(f"surrogate + fallback, check against the model's budget: {t_sur * 1e3:.1f} ms per step, {nfb} fallback pairs")
    # the network alone (every pair), timed with HIP events around its kernels
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    carb = [i for i, g in zip(ids, w5.grains) if g.composition == "carbonaceous"]
    parts = radius_groups(w5.grains, "carbonaceous", args.radius_groups)
    jn = {len(p): torch.empty((w5.n_cells, len(p), w5.n_lambda), dtype=torch.float32, device="cuda:0")
          for p in parts}

    def net_pass():
        # one composition: each range's network over its radii
        for p in parts:
            nets[p[0][0]].hsd_sur_predict(u, [ids[i] for i, _ in p], jn[len(p)], None, stream)

    net_pass()
    torch.cuda.synchronize()
    ev0.record(stream)
    net_pass()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_net = ev0.elapsed_time(ev1) * 1e-3
    del jn
    # accuracy on a seeded 1% sample of the pairs, against the plain GPU solve
    jp = jsu.view(n_pairs, -1).index_select(0, idx).cpu().numpy()
    err = _band_error(jp, jr, w5.lam_cm)
    flags = dsu.view(n_pairs, 4)[:, 3].index_select(0, idx).cpu().numpy().astype(np.int64)
    by_sur = (flags & 8) != 0
    log(f"1% sample: band error max {err.max():.4f} (surrogate pairs {err[by_sur].max() if by_sur.any() else 0:.4f}), "
        f"median {np.median(err):.5f}")
    # the tolerance trade-off: fewer fallbacks, larger errors
    sweep = []
    for tol in (0.02, 0.05):
        t_tol, nfb_tol = timed(lambda: ctx.hsd_solve_surrogate(u, ids, surs, jsu, dsu, tol=tol, check=hsd.CHECK_MODEL,
                                                               stream=stream), 1)
        e_tol = _band_error(jsu.view(n_pairs, -1).index_select(0, idx).cpu().numpy(), jr, w5.lam_cm)
        sweep.append({"tol": tol, "solves_per_s": n_pairs / t_tol, "speedup_vs_plain": t_plain / t_tol,
                      "fallback_fraction": nfb_tol / n_pairs, "sample_band_error_max": float(e_tol.max()),
                      "sample_band_error_p99": float(np.quantile(e_tol, 0.99))})
        log(f"tol {tol}: {t_tol * 1e3:.1f} ms, fallback {nfb_tol / n_pairs:.3f}, max band error {e_tol.max():.4f}")
    half_pairs = w5.n_cells * len(carb)
    out_bytes = half_pairs * w5.n_lambda * 4
    line = {"metric": METRIC, "value": n_pairs / t_sur, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": t_sur * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16 matmul + f32/f64 fallback", "data": "synthetic",
            "config": {"workload": "c5_surrogate", "cells": w5.n_cells, "grains": G, "n_lambda": w5.n_lambda,
                       "tol": 0.01, "check": "emitted vs the predicted absorbed power of the plain model",
                       "networks_per_composition": args.radius_groups},
            "plain_solves_per_s": n_pairs / t_plain, "speedup_vs_plain": t_plain / t_sur,
            "fallback_fraction": nfb / n_pairs,
            "check_against_absorbed": {"tol": 0.01, "solves_per_s": n_pairs / t_abs,
                                       "speedup_vs_plain": t_plain / t_abs, "fallback_fraction": nfb_abs / n_pairs,
                                       "sample_band_error_max": float(e_abs.max()),
                                       "sample_band_error_p99": float(np.quantile(e_abs, 0.99))},
            "sample_band_error": {"pairs": int(samp.shape[0]), "max": float(err.max()),
                                  "p99": float(np.quantile(err, 0.99)), "median": float(np.median(err)),
                                  "max_surrogate_pairs": float(err[by_sur].max()) if by_sur.any() else 0.0,
                                  "reference": "plain GPU solve (matches the FP64 oracle to 1e-4)"},
            "roofline": {"bound": "hbm", "kernel": "surrogate inference, one composition (network alone)",
                         "achieved": out_bytes / t_net / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": out_bytes / t_net / 8e12, "traffic": None, "kernel_ms": t_net * 1e3,
                         "bytes_per_launch": out_bytes},
            "tol_sweep": sweep,
            "training": report}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_batched")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cells", type=int, default=48)
    ap.add_argument("--eager", action="store_true", help="time hsd_solve calls instead of plan replays")
    ap.add_argument("--retune", action="store_true", help="time the launch configurations again")
    ap.add_argument("--contract", choices=("bf16x3", "fp32"), default="bf16x3",
                    help="emission contraction: three BF16 products of split operands, or FP32")
    ap.add_argument("--no-persistent", action="store_true",
                    help="launch every class as an ordinary grid (what a concurrent plan launches; for counter runs)")
    ap.add_argument("--train-steps", type=int, default=60000, help="surrogate training steps per network")
    ap.add_argument("--radius-groups", type=int, default=4,
                    help="surrogate networks per composition, each for one range of consecutive radii")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")     # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path "
              f"(its sharding is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.workload in ("c4_train", "c5_surrogate"):
        bench_surrogate(args)
        return

    cpu = None
    if not args.no_cpu_baseline:
        cpu, samples = cpu_baseline(args.workload, args.cpu_cells)
        print(f"cpu baseline: {cpu['value']:.1f} solves/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch
    from paper_1311_4627_amd import autotune, hsd

    w = synth.workload(args.workload)
    ctx = hsd.Context(w.lam_cm, device=0)
    ctx.hsd_set_contract(hsd.CONTRACT_FP32 if args.contract == "fp32" else hsd.CONTRACT_BF16X3)
    t0 = time.perf_counter()
    ids = [ctx.add_grain(g) for g in w.grains]
    setup_s = time.perf_counter() - t0
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells)
    ud = torch.tensor(u, device="cuda:0")
    j = torch.empty((w.n_cells, len(ids), w.n_lambda), dtype=torch.float32, device="cuda:0")
    diag = torch.empty((w.n_cells, len(ids), 4), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    print(f"setup {setup_s:.2f} s for {len(ids)} grains; {w.n_pairs} pairs per step", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tuned = autotune.tune(ctx, ud, ids, cache_path=TUNE_CACHE, force=args.retune)
    tune_s = time.perf_counter() - t0
    print(f"launch configuration ({'cached' if tuned['cached'] else 'timed'} in {tune_s:.1f} s): {tuned['cfg']}",
          file=sys.stderr, flush=True)
    # the configuration the timed launches use: a concurrent plan launches
    # every class as an ordinary grid
    launched = [dict(c) for c in tuned["cfg"]]
    if args.no_persistent or not args.eager:
        for c in launched:
            c["persistent"] = 0
        for cls, c in enumerate(launched):
            ctx.hsd_set_class_cfg(cls, **c)

    plan = None
    if not args.eager:
        plan = ctx.hsd_plan_create(ud, ids, j, diag, flags=hsd.PLAN_TIMING | hsd.PLAN_CONCURRENT)

    def step():
        if plan is not None:
            plan.hsd_plan_launch(stream)
        else:
            ctx.hsd_solve(ud, ids, j, diag, stream)

    for _ in range(args.warmup):
        step()
    ctx.hsd_sync()
    ctx.hsd_set_timing(True)
    phase = np.zeros(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        # waits on the step's own end event only
        phase += plan.hsd_plan_phase_ms() if plan is not None else ctx.hsd_phase_ms()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.hsd_set_timing(False)
    ctx.hsd_sync()
    ms_step = elapsed / args.steps * 1e3
    phase /= args.steps

    # the size-distribution convolution (a post-processing pass over j, not
    # part of the step): HBM-bound, reads j once and writes one spectrum per cell
    sizedist = None
    if args.workload == "c2_batched":
        radii = np.array([g.radius_cm for g in w.grains])
        out = torch.empty((w.n_cells, w.n_lambda), dtype=torch.float64, device="cuda:0")
        ctx.hsd_size_convolve(j, synth.size_weights(radii), out, stream=stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        ctx.hsd_size_convolve(j, synth.size_weights(radii), out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) * 1e-3
        nbytes = j.numel() * 4 + out.numel() * 8
        sizedist = {"ms": t * 1e3, "GB_per_s": nbytes / t / 1e9, "frac_of_hbm_peak": nbytes / t / 8e12}
        del out

    rates_per_step = 0
    for gi, g in zip(ids, w.grains):
        rates_per_step += count_rates(ctx.hsd_grain_tables(gi), w.lam_cm, g) * w.n_cells
    achieved = rates_per_step / (phase[0] * 1e-3)
    line = {
        "metric": METRIC,
        "value": w.n_pairs / (ms_step * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": w.n_cells, "grains": len(ids), "n_lambda": w.n_lambda,
                   "bins": f"{max(g.n_bins for g in w.grains)}..{min(g.n_bins for g in w.grains)} "
                           f"(sum {sum(g.n_bins for g in w.grains)})",
                   "launch": "eager" if plan is None else "plan (HIP graphs, concurrent classes)",
                   "contraction": args.contract,
                   "class_cfg": launched},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": EXP2_PEAK / 1e12, "unit": "Texp2/s",
                     "frac": achieved / EXP2_PEAK, "traffic": recorded_traffic(),
                     "kernel": "fused rates/recursion (k_solve)", "kernel_ms": phase[0],
                     "rates_per_launch": rates_per_step},
        "phases_ms": {"solve": phase[0], "contract": phase[1], "diag": phase[2]},
        "setup_s": setup_s,
        "tune_s": tune_s,
        "size_convolution": sizedist,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
        # the same sampled pairs, solved in the timed run, against the oracle
        line["oracle_error"] = oracle_error(j, samples)
        print(f"oracle check: {line['oracle_error']}", file=sys.stderr, flush=True)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
