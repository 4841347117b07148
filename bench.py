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
It runs before anything touches the GPU.
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
EXP2_PEAK = 157.3e12 / 2 / 4                 # v_exp_f32 per second: a quarter of the FP32 FMA rate
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve_c2_hbm_traffic.md")
TUNE_CACHE = os.path.join(ROOT, "paper_1311_4627_amd", "tuned.json")
SOLVER_SOURCES = ["paper_1311_4627_amd/csrc/hsd_solve.hip", "paper_1311_4627_amd/csrc/hsd_index.h",
                  "paper_1311_4627_amd/csrc/hsd_internal.h"]


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
    for c in range(len(cells)):
        oracle.solve_pair(u[c], g, w.lam_cm)
    return time.perf_counter() - t0, len(cells)


def cpu_baseline(name: str, cells_per_grain: int) -> dict:
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
    return {"value": rate, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{cells_per_grain} seeded cells x {len(w.grains)} radii of {name} "
                      f"({pairs} pairs, {busy:.1f} core-s of solve work, {wall:.1f} s wall incl. per-grain setup)"}


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
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a design note, "
              f"not part of this build", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, args.cpu_cells)
        print(f"cpu baseline: {cpu['value']:.1f} solves/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch
    from paper_1311_4627_amd import autotune, hsd

    w = synth.workload(args.workload)
    ctx = hsd.Context(w.lam_cm, device=0)
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
                   "class_cfg": tuned["cfg"]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": EXP2_PEAK / 1e12, "unit": "Texp2/s",
                     "frac": achieved / EXP2_PEAK, "traffic": recorded_traffic(),
                     "kernel": "fused rates/recursion (k_solve)", "kernel_ms": phase[0],
                     "rates_per_launch": rates_per_step},
        "phases_ms": {"solve": phase[0], "contract": phase[1], "diag": phase[2]},
        "setup_s": setup_s,
        "tune_s": tune_s,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
