"""Benchmark: emissivity solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload c5_surrogate | c2_batched | c3_uneven | c4_train]
                    [--no-cpu-baseline] [--exp2-rate] [--copy-calibration]

Default workload: the large surrogate workload, 262,144 cells (batched-
generator fields) x 64 radii x 2 compositions = 33,554,432 (cell, grain)
pairs on 500 wavelengths, the largest configuration that fits one GPU.  A
step is one solve of that whole batch:

* plain path (the line's `value`): the fused rates/recursion kernels, the
  emission contraction and the diagnostics for every pair, replayed from a
  plan (HIP graphs, solver classes as parallel branches, each smaller
  class's spectra contracted on its branch as soon as its solve ends),
  launch configuration from the autotuner's cache;
* table method (the cheap alternative the surrogate is measured against):
  plain spectra of one reference field shape at 57 log-spaced field
  strengths per grain, interpolated in log U and scaled by each pair's
  absorbed power, timed over the whole batch, with its band error;
* surrogate path: the networks (loaded from the committed checkpoints under
  paper_1311_4627_amd/weights/, trained by `bench.py --workload c4_train
  --save ...`), the in-kernel energy check at 1% and the plain solve on every
  flagged pair, reported as solves/s, speed-up over the plain path and
  fallback fraction.  The check compares each pair's emitted power with the
  table's energy budget (each node spectrum's emitted per absorbed power,
  interpolated at the cell's field strength): a reference made by plain
  solves alone.  The same path with the check against the network's own
  predicted budget, and against the absorbed power itself, is reported
  beside it.

Fields are resident in HBM before the timed region; spectra stay on the
device.  W untimed warm-up steps, then K timed steps of each path.  Prints
one JSON line.

Accuracy (both against the FP64 oracle, on a seeded sub-sample of the seeded
1% sample of the pairs): the plain path's largest relative error on j_lambda
(over wavelengths within 1e-10 of each spectrum's maximum; bar 1e-4) and the
surrogate path's band-integrated error (32 bands, bands holding >= 1e-3 of
the emitted power; bar 2%).  The surrogate's band error is also given on the
whole 1% sample against the plain GPU solve.

Roofline (the dominant kernel: the fused rates/recursion solver, timed with
HIP events on its stream inside the timed steps; the span of its four class
launches, which the smaller classes' contractions share while the largest
class still solves): the solver is bound by vector-ALU issue.  Algorithmic work per on-grid upward rate (a transition
whose photon wavelength lies on the grid): the log-grid index and the
log-log interpolation (six single-precision and integer operations), one
exponential (issued at half the lane rate on gfx950: two lane-cycles) and
the double-precision product-accumulate into the inflow sums (one): nine
lane-cycles.  Peak: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane-cycles/s.
The exponential alone (one per rate, 19.66e12/s: `--exp2-rate` measures the
device's rate) is reported beside it.  HBM traffic comes from the rocprofv3
FETCH_SIZE / WRITE_SIZE summary under profiles/ while the solver sources hash
to the value recorded there.

The CPU baseline is the FP64 oracle on the host: per-grain setup of the
sampled grains first (not timed, as the GPU's per-grain precompute is not),
then the sampled pairs solved by 16 worker processes (the machine's CPU share),
timed by the wall clock.  It runs before anything touches the GPU.
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
BAND_TOL = 0.02                              # surrogate bar on band-integrated j
LANE_RATE = 256 * 64 * 2.4e9                 # VALU lane-cycles per second (non-packed issue)
LANE_CYCLES_PER_RATE = 9                     # per on-grid rate: 6 index/interpolation + 2 exp2 + 1 FP64 fma
EXP2_RATE = LANE_RATE / 2                    # v_exp_f32 per second (half the lane rate on gfx950)
HBM_PEAK = 8.0e12
CPU_PROCS = 16
TUNE_CACHE = os.path.join(ROOT, "paper_1311_4627_amd", "tuned.json")
WEIGHTS_DIR = os.path.join(ROOT, "paper_1311_4627_amd", "weights")
# the solver kernel's own sources (a traffic summary is valid while they are unchanged)
SOLVER_SOURCES = ["paper_1311_4627_amd/csrc/hsd_solve.hip", "paper_1311_4627_amd/csrc/hsd_index.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def solver_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SOLVER_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str):
    """HBM bytes per solve phase from the committed counter summary of this
    workload, or None when it is missing or was taken on other solver sources."""
    path = os.path.join(ROOT, "profiles", f"solve_{workload.split('_')[0]}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("solver_sources_sha256_16:"):
            vals["hash"] = line.split(":", 1)[1].strip()
        if line.startswith("solve_phase_hbm_bytes_per_step:"):
            vals["bytes"] = float(line.split(":", 1)[1].strip())
    if vals.get("hash") != solver_hash() or "bytes" not in vals:
        return None
    return vals["bytes"]


# ---- the CPU leg: the FP64 oracle on sampled pairs ----------------------------------

def _oracle_setup_task(args):
    name, gi = args
    import oracle
    w = synth.workload(name, n_cells=1)
    return gi, oracle.grain_setup(w.grains[gi], w.lam_cm)


def _oracle_solve_task(args):
    name, gi, cells, n_total = args
    import oracle
    w = synth.workload(name, n_cells=1)
    u = make_fields(w.lam_cm, w.field_recipe, n_total, cells=np.asarray(cells))
    t0 = time.perf_counter()
    js = [oracle.solve_pair(u[c], w.grains[gi], w.lam_cm)[1] for c in range(len(cells))]
    return time.perf_counter() - t0, gi, list(cells), np.stack(js)


def oracle_pairs(name: str, n_total: int, pairs_by_grain: dict):
    """The FP64 oracle's spectra of the given pairs ({grain: [cells]}) and the
    CPU baseline record.  Grain setups run first in a pool and are handed to
    the solving workers (not timed); the solves are timed by the wall clock."""
    from oracle import model as om
    w = synth.workload(name, n_cells=1)
    grains = sorted(pairs_by_grain)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(CPU_PROCS) as pool:
        setups = pool.map(_oracle_setup_task, [(name, gi) for gi in grains], chunksize=1)
    setup_s = time.perf_counter() - t0
    for gi, s in setups:                         # the solving workers inherit these through fork
        om.preload_setup(w.grains[gi], w.lam_cm, s)
    # a few cells per task, longest grains first, so that the pool stays busy
    tasks = []
    for gi in sorted(grains, key=lambda g: -w.grains[g].n_bins):
        cells = sorted(pairs_by_grain[gi])
        for k in range(0, len(cells), 8):
            tasks.append((name, gi, cells[k:k + 8], n_total))
    t0 = time.perf_counter()
    with ctx.Pool(CPU_PROCS) as pool:
        res = pool.map(_oracle_solve_task, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    busy = sum(r[0] for r in res)
    n = sum(len(r[2]) for r in res)
    rec = {"value": n / wall, "unit": "solves/s", "cores": CPU_PROCS, "kind": "oracle",
           "sample": f"{n} seeded pairs of {name} over {len(grains)} grains, solved by {CPU_PROCS} processes "
                     f"in {wall:.1f} s wall ({busy:.1f} process-s); per-grain setup {setup_s:.1f} s not timed"}
    spectra = {}
    for _, gi, cells, js in res:
        for c, jr in zip(cells, js):
            spectra[(c, gi)] = jr
    return rec, spectra


def j_rel_err(j: np.ndarray, jref: np.ndarray) -> float:
    """Largest |j / j_ref - 1| over the wavelengths where j_ref is at least
    1e-10 of the spectrum's maximum (the range the 1e-4 bar covers)."""
    if jref.max() <= 0.0:
        return 0.0 if np.all(j == 0.0) else math.inf
    m = jref >= 1e-10 * jref.max()
    return float(np.max(np.abs(j[m] / jref[m] - 1.0))) if np.any(m) else 0.0


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


def roofline(rates: int, solve_ms: float, traffic):
    """The solver phase against the vector-ALU issue bound (see the module
    docstring); the exponential's own fraction beside it."""
    t = solve_ms * 1e-3
    achieved = rates * LANE_CYCLES_PER_RATE / t
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": LANE_RATE / 1e12, "unit": "Tlane-cycle/s",
            "frac": achieved / LANE_RATE, "traffic": traffic,
            "kernel": "fused rates/recursion solver (k_solve, all bin classes)", "kernel_ms": solve_ms,
            "rates_per_launch": rates, "lane_cycles_per_rate": LANE_CYCLES_PER_RATE,
            "exp2": {"achieved": rates / t / 1e12, "peak": EXP2_RATE / 1e12, "unit": "Texp2/s",
                     "frac": rates / t / EXP2_RATE}}


def radius_groups(grains, comp: str, n_groups: int):
    """The composition's grains split into n_groups ranges of consecutive
    radii (the workloads list radii in increasing order): (index, grain)
    lists, one network each."""
    sel = [(i, g) for i, g in enumerate(grains) if g.composition == comp]
    G = len(sel)
    return [sel[q * G // n_groups:(q + 1) * G // n_groups] for q in range(n_groups)]


# the table method: nodes every 1/8 dex of U over the range of the generators' fields (U 0.1 .. 1e5,
# with a jitter of up to 30% per component), the reference shape being the unjittered field at U = 1
TABLE_LOG10U = (-1.5, 5.5)
TABLE_NODES = 57


def table_method(torch, ctx, w, ids, u, j, stream=None):
    """Table-method spectra of every (cell, grain) pair of u x ids into j; returns
    the seconds the table build took and a call that evaluates the table again.
    The table is also set as the energy budget of the surrogate's table check."""
    from synth.fields import FieldRecipe
    u_ref = torch.tensor(make_fields(w.lam_cm, FieldRecipe(0, (1.0, 1.0), 0.0, None), 1)[0], device="cuda:0")
    lo, hi = TABLE_LOG10U
    table = torch.empty((len(ids), TABLE_NODES, w.n_lambda), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.hsd_table_build(ids, u_ref, lo, hi, table, stream)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ctx.hsd_set_energy_budget(ids, u_ref, lo, hi, table, stream)
    ctx.hsd_table_eval(u, ids, u_ref, lo, hi, table, j, stream)
    return build_s, (lambda: ctx.hsd_table_eval(u, ids, u_ref, lo, hi, table, j, stream))


def train_surrogates(torch, hsd, ctx, w4, ids, steps, batch, lr, log, n_groups=4, band_weight=0.0, save_dir=None):
    """Per composition and range of radii: plain-solve the training cells for
    those radii, build inputs and targets, fit the statistics and train one
    network; then the held-out band errors.  Returns the networks keyed by
    grain index and a report per composition.  With save_dir, each network is
    written there as a weights-only checkpoint, listed in manifest.json."""
    from synth import surrogate as ssur
    nets, report = {}, {}
    manifest = {"workload": "c4_train", "steps": steps, "batch": batch, "lr": lr, "loss_band_weight": band_weight,
                "networks": []}
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
            sur.hsd_sur_set_loss(band_weight)
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
            # the cheap method the surrogate replaces: the table method (hsd_table_*),
            # plain spectra of the reference field shape at log-spaced U, interpolated
            # in log U and scaled by the pair's own absorbed power
            jt = torch.empty_like(jr)
            table_method(torch, ctx, w4, sel, uh, jt)
            terr = _band_error(jt.cpu().numpy().reshape(-1, w4.n_lambda), jr.cpu().numpy().reshape(-1, w4.n_lambda),
                               w4.lam_cm)
            del X, Y, A, jt, jr, jp, dr, dp
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
            if save_dir:
                fname = f"{comp}_{len(groups) - 1}.hsdsur"
                sur.hsd_surrogate_save(os.path.join(save_dir, fname), weights_only=True)
                manifest["networks"].append({"file": fname, "composition": comp,
                                             "grains": [i for i, _ in part], "radii_A": [round(r0, 2), round(r1, 2)],
                                             "heldout_band_err_max": float(err.max())})
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
    if save_dir:
        with open(os.path.join(save_dir, "manifest.json"), "w") as f:
            json.dump(manifest, f, indent=1)
    return nets, report


def load_networks(hsd, ctx, w, weights_dir: str):
    """The committed networks (weights-only checkpoints listed in
    manifest.json), one per range of radii: a list giving each grain of w its
    network, and the manifest."""
    man_path = os.path.join(weights_dir, "manifest.json")
    if not os.path.exists(man_path):
        raise SystemExit(f"{man_path} is missing: train with `bench.py --workload c4_train --save {weights_dir}`")
    with open(man_path) as f:
        man = json.load(f)
    surs = [None] * len(w.grains)
    for ent in man["networks"]:
        sur = hsd.Surrogate(ctx)
        sur.hsd_surrogate_load(os.path.join(weights_dir, ent["file"]))
        for gi in ent["grains"]:
            if w.grains[gi].composition != ent["composition"]:
                raise SystemExit(f"{ent['file']}: grain {gi} is not {ent['composition']}")
            surs[gi] = sur
    if any(s is None for s in surs):
        raise SystemExit("the manifest leaves grains without a network")
    return surs, man


def timed_steps(torch, fn, warmup: int, steps: int):
    """W untimed calls, then the wall time of K calls between device-wide
    synchronisations; returns (seconds per call, last result)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1), out


def plain_plan(hsd, autotune, ctx, ud, ids, j, d, retune=False):
    """The autotuned configuration (cached), every class as an ordinary grid,
    as one plan with phase timing and concurrent classes."""
    tuned = autotune.tune(ctx, ud, ids, cache_path=TUNE_CACHE, force=retune)
    launched = [dict(c, persistent=0) for c in tuned["cfg"]]
    for cls, c in enumerate(launched):
        ctx.hsd_set_class_cfg(cls, **c)
    plan = ctx.hsd_plan_create(ud, ids, j, d, flags=hsd.PLAN_TIMING | hsd.PLAN_CONCURRENT)
    launched = {"classes": launched, "contract_waves": ctx.hsd_get_contract_waves()}
    return plan, launched, tuned["cached"]


def timed_plan(torch, plan, stream, warmup, steps):
    """Plan replays: W untimed, then K timed; mean phase times from the
    plan's HIP events (recorded on the replay stream)."""
    for _ in range(warmup):
        plan.hsd_plan_launch(stream)
    torch.cuda.synchronize()
    phase = np.zeros(3)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.hsd_plan_launch(stream)
        phase += plan.hsd_plan_phase_ms()       # waits on this replay's end event only
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, phase / steps


def bench_c5(args):
    """The default line: plain and surrogate paths on the 33.5M-pair workload."""
    name = "c5_surrogate"
    w = synth.workload(name)
    G, L, n_cells = len(w.grains), w.n_lambda, w.n_cells
    n_pairs = n_cells * G
    # the seeded 1% sample of the pairs, and the oracle's sub-sample of it
    rng = np.random.default_rng(4627005)
    samp = np.sort(rng.choice(n_pairs, n_pairs // 100, replace=False))
    sub = np.sort(np.random.default_rng(4627105).choice(samp, args.oracle_pairs, replace=False))
    by_grain = {}
    for p in sub:
        by_grain.setdefault(int(p % G), []).append(int(p // G))
    cpu = spectra = None
    if not args.no_cpu_baseline:
        cpu, spectra = oracle_pairs(name, n_cells, by_grain)
        log(f"cpu baseline: {cpu['value']:.1f} solves/s ({cpu['sample']})")

    import torch
    from paper_1311_4627_amd import autotune, hsd
    ctx = hsd.Context(w.lam_cm, device=0)
    t0 = time.perf_counter()
    ids = [ctx.add_grain(g) for g in w.grains]
    setup_s = time.perf_counter() - t0
    surs, man = load_networks(hsd, ctx, w, args.weights)
    log(f"setup {setup_s:.2f} s for {G} grains; {len(man['networks'])} networks from {args.weights}")
    ud = torch.tensor(make_fields(w.lam_cm, w.field_recipe, n_cells), device="cuda:0")
    stream = torch.cuda.current_stream()
    jpl = torch.empty((n_cells, G, L), dtype=torch.float32, device="cuda:0")
    dpl = torch.empty((n_cells, G, 4), dtype=torch.float32, device="cuda:0")
    plan, launched, cached = plain_plan(hsd, autotune, ctx, ud, ids, jpl, dpl, args.retune)
    log(f"launch configuration {launched} (cached: {cached})")
    t_plain, phase = timed_plan(torch, plan, stream, args.warmup, args.steps)
    log(f"plain: {t_plain * 1e3:.1f} ms per step (solve {phase[0]:.1f}, contraction {phase[1]:.1f}, "
        f"diagnostics {phase[2]:.1f})")
    jsu = torch.empty_like(jpl)
    dsu = torch.empty_like(dpl)

    def sur_step(check):
        return ctx.hsd_solve_surrogate(ud, ids, surs, jsu, dsu, tol=0.01, check=check, stream=stream)

    # the literal check against the absorbed power A, one step (its output is overwritten below)
    t_abs, nfb_abs = timed_steps(torch, lambda: sur_step(hsd.CHECK_ABSORBED), 1, 1)
    idx = torch.tensor(samp, device="cuda:0")
    jr_gpu = jpl.view(n_pairs, L).index_select(0, idx).cpu().numpy()
    e_abs = _band_error(jsu.view(n_pairs, L).index_select(0, idx).cpu().numpy(), jr_gpu, w.lam_cm)
    log(f"surrogate, check against A: {t_abs * 1e3:.1f} ms, {nfb_abs} fallback pairs")
    t_mod, nfb_mod = timed_steps(torch, lambda: sur_step(hsd.CHECK_MODEL), args.warmup, args.steps)
    e_mod = _band_error(jsu.view(n_pairs, L).index_select(0, idx).cpu().numpy(), jr_gpu, w.lam_cm)
    log(f"surrogate, check against the network's rho A: {t_mod * 1e3:.1f} ms per step, {nfb_mod} fallback pairs")
    # the table method over the whole batch (into the surrogate's buffer), its band error on the sample
    build_s, tab_eval = table_method(torch, ctx, w, ids, ud, jsu, stream)
    t_tab, _ = timed_steps(torch, tab_eval, 1, args.steps)
    e_tab = _band_error(jsu.view(n_pairs, L).index_select(0, idx).cpu().numpy(), jr_gpu, w.lam_cm)
    log(f"table method: {t_tab * 1e3:.1f} ms per step, sample band error median {np.median(e_tab):.4f} "
        f"max {e_tab.max():.4f}")
    # the surrogate path as measured: the check against the table's energy
    # budget (plain solves only, none of the networks' outputs)
    t_sur, nfb = timed_steps(torch, lambda: sur_step(hsd.CHECK_TABLE), args.warmup, args.steps)
    log(f"surrogate, check against the table budget: {t_sur * 1e3:.1f} ms per step, {nfb} fallback pairs")
    # accuracy: the 1% sample against the plain GPU solve; the sub-sample against the oracle
    jsp = jsu.view(n_pairs, L).index_select(0, idx).cpu().numpy()
    err = _band_error(jsp, jr_gpu, w.lam_cm)
    flags = dsu.view(n_pairs, 4)[:, 3].index_select(0, idx).cpu().numpy().astype(np.int64)
    by_sur = (flags & 8) != 0
    oracle_err = None
    if spectra is not None:
        pos = np.searchsorted(samp, sub)
        jr_o = np.stack([spectra[(int(p // G), int(p % G))] for p in sub])
        j_plain = jr_gpu[pos].astype(np.float64)
        worst = max(j_rel_err(j_plain[k], jr_o[k]) for k in range(len(sub)))
        e_or = _band_error(jsp[pos], jr_o, w.lam_cm)
        oracle_err = {"pairs": int(len(sub)), "plain_max_rel_err_j": worst, "tol": J_TOL,
                      "plain_within_tol": bool(worst <= J_TOL),
                      "surrogate_band_err": {"max": float(e_or.max()), "p99": float(np.quantile(e_or, 0.99)),
                                             "median": float(np.median(e_or)), "tol": BAND_TOL,
                                             "within_tol": bool(e_or.max() <= BAND_TOL)}}
        log(f"against the oracle ({len(sub)} pairs): plain j max rel err {worst:.2e}; surrogate band error "
            f"max {e_or.max():.4f}")
    # the networks alone over one composition (HBM-write bound), HIP events on the stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    carb = [g for g in range(G) if w.grains[g].composition == "carbonaceous"]
    groups = {}
    for g in carb:
        groups.setdefault(id(surs[g]), (surs[g], []))[1].append(g)
    jn = {n: torch.empty((n_cells, n, L), dtype=torch.float32, device="cuda:0")
          for n in {len(v[1]) for v in groups.values()}}

    def net_pass():
        for sur, gs in groups.values():
            sur.hsd_sur_predict(ud, [ids[g] for g in gs], jn[len(gs)], None, stream)

    net_pass()
    torch.cuda.synchronize()
    ev0.record(stream)
    net_pass()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_net = ev0.elapsed_time(ev1) * 1e-3
    del jn
    out_bytes = n_cells * len(carb) * L * 4
    rates = sum(count_rates(ctx.hsd_grain_tables(i), w.lam_cm, g) for i, g in zip(ids, w.grains)) * n_cells
    line = {
        "metric": METRIC, "value": n_pairs / t_plain, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_plain * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 rates, f64 sums and recursion, bf16x3 contraction",
        "data": "synthetic",
        "config": {"workload": name, "cells": n_cells, "grains": G, "n_lambda": L,
                   "bins": f"{max(g.n_bins for g in w.grains)}..{min(g.n_bins for g in w.grains)} "
                           f"(sum {sum(g.n_bins for g in w.grains)})",
                   "launch": "plan (HIP graphs, concurrent classes)", "class_cfg": launched,
                   "surrogate": {"networks": len(man["networks"]), "net": "33-256-256-256-501 GELU, bf16 matmul",
                                 "weights": os.path.relpath(args.weights, ROOT), "tol": 0.01,
                                 "check": "emitted vs A rho(t) (rho: the table's node spectra, emitted per "
                                          "absorbed power, interpolated in log U; plain solves only)"}},
        "roofline": roofline(rates, phase[0], recorded_traffic(name)),
        "phases_ms": {"solve": phase[0], "contract": phase[1], "diag": phase[2]},
        "surrogate_solves_per_s": n_pairs / t_sur, "speedup_vs_plain": t_plain / t_sur,
        "surrogate_ms_per_step": t_sur * 1e3, "fallback_fraction": nfb / n_pairs,
        "check_against_model": {"tol": 0.01, "solves_per_s": n_pairs / t_mod, "speedup_vs_plain": t_plain / t_mod,
                                "ms_per_step": t_mod * 1e3, "fallback_fraction": nfb_mod / n_pairs,
                                "reference": "rho A, rho the network's own predicted emitted/absorbed power",
                                "sample_band_error_max": float(e_mod.max())},
        "check_against_absorbed": {"tol": 0.01, "solves_per_s": n_pairs / t_abs, "speedup_vs_plain": t_plain / t_abs,
                                   "fallback_fraction": nfb_abs / n_pairs, "sample_band_error_max": float(e_abs.max())},
        "sample_band_error_vs_plain": {"pairs": int(samp.shape[0]), "max": float(err.max()),
                                       "p99": float(np.quantile(err, 0.99)), "median": float(np.median(err)),
                                       "max_surrogate_pairs": float(err[by_sur].max()) if by_sur.any() else 0.0},
        "oracle_error": oracle_err,
        "table_method": {"nodes": TABLE_NODES, "log10U": list(TABLE_LOG10U), "build_s": build_s,
                         "solves_per_s": n_pairs / t_tab, "ms_per_step": t_tab * 1e3,
                         "sample_band_error_vs_plain": {"max": float(e_tab.max()),
                                                        "p99": float(np.quantile(e_tab, 0.99)),
                                                        "median": float(np.median(e_tab))}},
        "surrogate_roofline": {"bound": "hbm", "kernel": "network inference, one composition", "unit": "GB/s",
                               "achieved": out_bytes / t_net / 1e9, "peak": HBM_PEAK / 1e9,
                               "frac": out_bytes / t_net / HBM_PEAK, "kernel_ms": t_net * 1e3,
                               "bytes_per_launch": out_bytes},
        "setup_s": setup_s,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    plan.close()
    del jpl, dpl, jsu, dsu, ud
    torch.cuda.empty_cache()
    if not args.no_c3:
        line["c3_uneven"] = plain_workload(torch, hsd, autotune, "c3_uneven", 1, 3)
        log(f"c3_uneven: {line['c3_uneven']['solves_per_s']:.4g} solves/s")
    print(json.dumps(line))


def plain_workload(torch, hsd, autotune, name, warmup, steps):
    """Plain solves/s of another workload (plan replays), as an extra key."""
    w = synth.workload(name)
    ctx = hsd.Context(w.lam_cm, device=0)
    ids = [ctx.add_grain(g) for g in w.grains]
    ud = torch.tensor(make_fields(w.lam_cm, w.field_recipe, w.n_cells), device="cuda:0")
    j = torch.empty((w.n_cells, len(ids), w.n_lambda), dtype=torch.float32, device="cuda:0")
    d = torch.empty((w.n_cells, len(ids), 4), dtype=torch.float32, device="cuda:0")
    plan, launched, _ = plain_plan(hsd, autotune, ctx, ud, ids, j, d)
    t, phase = timed_plan(torch, plan, torch.cuda.current_stream(), warmup, steps)
    plan.close()
    ctx.close()
    return {"cells": w.n_cells, "grains": len(ids), "pairs": w.n_pairs, "solves_per_s": w.n_pairs / t,
            "ms_per_step": t * 1e3, "steps": steps, "phases_ms": {"solve": phase[0], "contract": phase[1],
                                                                  "diag": phase[2]}}


def bench_plain(args):
    """The batched or uneven workload alone (plain path)."""
    name = args.workload
    w = synth.workload(name)
    cpu = spectra = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(4627)
        by_grain = {gi: sorted(rng.choice(w.n_cells, size=args.cpu_cells, replace=False).tolist())
                    for gi in range(len(w.grains))}
        cpu, spectra = oracle_pairs(name, w.n_cells, by_grain)
        log(f"cpu baseline: {cpu['value']:.1f} solves/s ({cpu['sample']})")
    import torch
    from paper_1311_4627_amd import autotune, hsd
    ctx = hsd.Context(w.lam_cm, device=0)
    ctx.hsd_set_contract(hsd.CONTRACT_FP32 if args.contract == "fp32" else hsd.CONTRACT_BF16X3)
    t0 = time.perf_counter()
    ids = [ctx.add_grain(g) for g in w.grains]
    setup_s = time.perf_counter() - t0
    ud = torch.tensor(make_fields(w.lam_cm, w.field_recipe, w.n_cells), device="cuda:0")
    j = torch.empty((w.n_cells, len(ids), w.n_lambda), dtype=torch.float32, device="cuda:0")
    diag = torch.empty((w.n_cells, len(ids), 4), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    log(f"setup {setup_s:.2f} s for {len(ids)} grains; {w.n_pairs} pairs per step")
    if args.eager:
        tuned = autotune.tune(ctx, ud, ids, cache_path=TUNE_CACHE, force=args.retune)
        classes = tuned["cfg"]
        if args.no_persistent:
            # the kernels and work order of the concurrent plan as eager calls (one dispatch per
            # class; counter collection runs the dispatches one at a time)
            classes = [dict(c, persistent=0) for c in classes]
            for cls, c in enumerate(classes):
                ctx.hsd_set_class_cfg(cls, **c)
        launched = {"classes": classes, "contract_waves": ctx.hsd_get_contract_waves()}
        for _ in range(args.warmup):
            ctx.hsd_solve(ud, ids, j, diag, stream)
        ctx.hsd_sync()
        ctx.hsd_set_timing(True)
        phase = np.zeros(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.hsd_solve(ud, ids, j, diag, stream)
            phase += ctx.hsd_phase_ms()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        phase /= args.steps
        ctx.hsd_set_timing(False)
        plan = None
    else:
        plan, launched, _ = plain_plan(hsd, autotune, ctx, ud, ids, j, diag, args.retune)
        t_step, phase = timed_plan(torch, plan, stream, args.warmup, args.steps)
    ctx.hsd_sync()
    log(f"{t_step * 1e3:.2f} ms per step (solve {phase[0]:.2f}, contraction {phase[1]:.2f}, diagnostics {phase[2]:.2f})")
    rates = sum(count_rates(ctx.hsd_grain_tables(i), w.lam_cm, g) for i, g in zip(ids, w.grains)) * w.n_cells
    line = {
        "metric": METRIC, "value": w.n_pairs / t_step, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"f32 rates, f64 sums and recursion, {args.contract} contraction",
        "data": "synthetic",
        "config": {"workload": name, "cells": w.n_cells, "grains": len(ids), "n_lambda": w.n_lambda,
                   "bins": f"{max(g.n_bins for g in w.grains)}..{min(g.n_bins for g in w.grains)} "
                           f"(sum {sum(g.n_bins for g in w.grains)})",
                   "launch": "eager" if plan is None else "plan (HIP graphs, concurrent classes)",
                   "class_cfg": launched},
        "roofline": roofline(rates, phase[0], recorded_traffic(name)),
        "phases_ms": {"solve": phase[0], "contract": phase[1], "diag": phase[2]},
        "setup_s": setup_s,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
        worst, n = 0.0, 0
        for gi, cells in sorted({gi: [c for (c, g) in spectra if g == gi] for gi in range(len(ids))}.items()):
            if not cells:
                continue
            got = j[:, gi].index_select(0, torch.tensor(cells, device="cuda:0")).cpu().numpy().astype(np.float64)
            for k, c in enumerate(cells):
                worst = max(worst, j_rel_err(got[k], spectra[(c, gi)]))
                n += 1
        line["oracle_error"] = {"pairs": n, "max_rel_err_j": worst, "tol": J_TOL, "within_tol": bool(worst <= J_TOL)}
        log(f"oracle check: {line['oracle_error']}")
    if name == "c2_batched":
        # the size-distribution convolution (a post-processing pass over j, not part of the step)
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
        line["size_convolution"] = {"ms": t * 1e3, "GB_per_s": nbytes / t / 1e9, "frac_of_hbm_peak": nbytes / t / HBM_PEAK}
    if plan is not None:
        plan.close()
    print(json.dumps(line))


def bench_c4(args):
    """Train every network of both compositions and report held-out errors."""
    import torch
    from paper_1311_4627_amd import hsd
    w4 = synth.workload("c4_train")
    ctx = hsd.Context(w4.lam_cm, device=0)
    ids = [ctx.add_grain(g) for g in w4.grains]
    if args.save:
        os.makedirs(args.save, exist_ok=True)
    nets, report = train_surrogates(torch, hsd, ctx, w4, ids, args.train_steps, 4096, 4e-3, log,
                                    args.radius_groups, args.band_weight, args.save)
    tot_pairs = sum(r["train_pairs"] for r in report.values())
    tot_s = sum(r["train_s"] for r in report.values())
    n_nets = sum(r["networks"] for r in report.values())
    line = {"metric": "surrogate training: samples per second (held-out band errors reported)",
            "value": args.train_steps * 4096 * n_nets / tot_s, "unit": "samples/s", "n_gpus": 1,
            "steps": args.train_steps, "warmup": 0, "ms_per_step": 1e3 * tot_s / (args.train_steps * n_nets),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 matmul, f32 master",
            "data": "synthetic", "config": {"workload": "c4_train", "train_pairs": tot_pairs,
                                            "net": "33-256-256-256-501 GELU",
                                            "networks_per_composition": args.radius_groups,
                                            "loss_band_weight": args.band_weight},
            "per_composition": report}
    print(json.dumps(line))


def exp2_rate():
    """The device's v_exp_f32 issue rate (a calibration of the roofline's
    exponential figure)."""
    import torch
    from paper_1311_4627_amd import hsd
    ctx = hsd.Context(synth.wavelength_grid_cm(500), device=0)
    r = ctx.hsd_measure_exp2()
    torch.cuda.synchronize()
    print(json.dumps({"exp2_per_s": r, "lane_rate": LANE_RATE, "per_lane_cycle": r / LANE_RATE,
                      "assumed_peak": EXP2_RATE}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5_surrogate",
                    choices=("c5_surrogate", "c2_batched", "c3_uneven", "c4_train"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cells", type=int, default=48, help="c2/c3: oracle cells per grain")
    ap.add_argument("--oracle-pairs", type=int, default=2048, help="c5: oracle pairs (from the 1%% sample)")
    ap.add_argument("--no-c3", action="store_true", help="c5: skip the uneven workload's extra key")
    ap.add_argument("--weights", default=WEIGHTS_DIR, help="c5: directory of the trained networks")
    ap.add_argument("--eager", action="store_true", help="c2/c3: time hsd_solve calls instead of plan replays")
    ap.add_argument("--retune", action="store_true", help="time the launch configurations again (cache ignored)")
    ap.add_argument("--no-persistent", action="store_true",
                    help="c2/c3 eager: every class as an ordinary grid (the plan's kernels, for counter runs)")
    ap.add_argument("--contract", choices=("bf16x3", "fp32"), default="bf16x3",
                    help="c2/c3: emission contraction: three BF16 products of split operands, or FP32")
    ap.add_argument("--train-steps", type=int, default=60000, help="c4: training steps per network")
    ap.add_argument("--radius-groups", type=int, default=4,
                    help="c4: networks per composition, each for one range of consecutive radii")
    ap.add_argument("--band-weight", type=float, default=0.0,
                    help="c4: weight of the band-weighted loss (0 = plain mean squared error)")
    ap.add_argument("--save", default=None, help="c4: directory for the trained networks")
    ap.add_argument("--exp2-rate", action="store_true", help="only measure the device's exp2 issue rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        log(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path "
            f"(its sharding is described in the design notes)")
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")     # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return
    if args.exp2_rate:
        exp2_rate()
        return
    if args.workload == "c4_train":
        bench_c4(args)
    elif args.workload == "c5_surrogate":
        bench_c5(args)
    else:
        bench_plain(args)


if __name__ == "__main__":
    main()
