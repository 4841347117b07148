"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 steps (identical FP64 rates in) <= 1e-6 relative on P over bins
with P_ref >= 1e-250; end to end <= 1e-4 relative on j_lambda over wavelengths
with j_ref >= 1e-10 max j_ref.  Inputs are the seeded synthetic workloads.
"""

import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import model as om
from synth.fields import make_fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

J_TOL = 1e-4
P64_TOL = 1e-6


def j_rel_err(j, jref):
    if jref.max() <= 0.0:
        return 0.0 if np.all(j == 0.0) else math.inf
    m = jref >= 1e-10 * jref.max()
    return float(np.max(np.abs(j[m] / jref[m] - 1.0))) if np.any(m) else 0.0


@pytest.fixture(scope="module")
def hsd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4627_amd import hsd as h
    return h


@pytest.fixture(scope="module")
def c1(hsd):
    w = synth.workload("c1_tiny")
    ctx = hsd.Context(w.lam_cm)
    gid = ctx.add_grain(w.grains[0])
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells)
    return w, ctx, gid, u


def test_grain_tables_match_oracle(hsd):
    lam = synth.wavelength_grid_cm(500)
    grains = [synth.make_grain("carbonaceous", 3.5e-8, lam), synth.make_grain("carbonaceous", 250e-8, lam),
              synth.make_grain("silicate", 2500e-8, lam), synth.make_grain("silicate", 20e-8, lam)]
    ctx = hsd.Context(lam)
    for g in grains:
        gid = ctx.add_grain(g)
        E, dE, T, cool = ctx.hsd_grain_tables(gid)
        s = oracle.grain_setup(g, lam)
        print(f"grain a={g.radius_cm:.2e} n={g.n_bins}", flush=True)
        assert np.max(np.abs(E / s.E - 1)) < 1e-13
        assert np.max(np.abs(dE / s.dE - 1)) < 1e-12
        assert np.max(np.abs(T / s.T - 1)) < 1e-12
        assert cool[0] == 0.0
        assert np.max(np.abs(cool[1:] / s.cool[1:] - 1)) < 1e-9


@pytest.mark.parametrize("nb", [16, 128, 256, 512, 1024])
def test_from_rates_matches_oracle_recursion(hsd, c1, nb):
    _, ctx, _, _ = c1
    rng = np.random.default_rng(nb)
    n_pairs = 5                                    # ragged against every block shape
    A = np.zeros((n_pairs, nb, nb))
    cool = np.zeros((n_pairs, nb))
    for p in range(n_pairs):
        A[p] = np.tril(10.0 ** rng.uniform(-8, 2, size=(nb, nb)), k=-1)
        A[p][rng.uniform(size=(nb, nb)) < 0.3] = 0.0
        A[p] = np.tril(A[p], k=-1)
        cool[p, 1:] = 10.0 ** rng.uniform(-6, 0, size=nb - 1)
    Ad = torch.tensor(A, device="cuda")
    cd = torch.tensor(cool, device="cuda")
    Pd = torch.empty((n_pairs, nb), dtype=torch.float64, device="cuda")
    ctx.hsd_solve_from_rates(Ad, cd, Pd)
    ctx.hsd_sync()
    P = Pd.cpu().numpy()
    for p in range(n_pairs):
        Pref, _, nres = om.recursion(om.b_matrix_recurrence(A[p]), cool[p])
        m = Pref >= 1e-250
        err = np.max(np.abs(P[p][m] / Pref[m] - 1.0))
        print(f"nb={nb} pair={p} rescales={nres} max rel err P={err:.2e}", flush=True)
        assert err < P64_TOL
        assert np.all(P[p][~m] < 1e-240)


def test_from_rates_physical_c1(hsd, c1):
    w, ctx, gid, u = c1
    s = oracle.grain_setup(w.grains[0], w.lam_cm)
    cells = [0, 9, 33, 63]
    A = np.stack([om.heating_matrix(u[c], s) for c in cells])
    cool = np.tile(s.cool, (len(cells), 1))
    Pd = torch.empty((len(cells), 256), dtype=torch.float64, device="cuda")
    ctx.hsd_solve_from_rates(torch.tensor(A, device="cuda"), torch.tensor(cool, device="cuda"), Pd)
    ctx.hsd_sync()
    P = Pd.cpu().numpy()
    for i, c in enumerate(cells):
        Pref, _, _ = om.recursion(om.b_matrix_recurrence(A[i]), s.cool)
        m = Pref >= 1e-250
        err = np.max(np.abs(P[i][m] / Pref[m] - 1.0))
        print(f"c1 cell {c}: FP64-step max rel err {err:.2e}", flush=True)
        assert err < P64_TOL


@pytest.mark.parametrize("contract", ["bf16x3", "fp32"])
def test_solve_c1_end_to_end(hsd, c1, contract):
    # both emission contractions against the oracle: the split-BF16 products
    # (the default) and FP32 products on the matrix cores
    w, ctx, gid, u = c1
    n = w.n_cells
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((n, 1, w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((n, 1, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_set_contract(hsd.CONTRACT_FP32 if contract == "fp32" else hsd.CONTRACT_BF16X3)
    try:
        ctx.hsd_solve(ud, [gid], j, diag)
        ctx.hsd_sync()
    finally:
        ctx.hsd_set_contract(hsd.CONTRACT_BF16X3)
    j = j.cpu().numpy()[:, 0, :].astype(np.float64)
    diag = diag.cpu().numpy()[:, 0, :].astype(np.float64)
    worst = 0.0
    for c in range(n):
        P, jr, d = oracle.solve_pair(u[c], w.grains[0], w.lam_cm, with_diag=True)
        e = j_rel_err(j[c], jr)
        worst = max(worst, e)
        assert e < J_TOL, (c, e)
        assert abs(diag[c, 0] / d["absorbed"] - 1) < 1e-6
        assert abs(diag[c, 1] / d["emitted"] - 1) < J_TOL
        assert abs(diag[c, 2] / d["A_rep"] - 1) < J_TOL
        assert int(diag[c, 3]) & 1 == 0
    print(f"c1 end-to-end ({contract} contraction) worst j rel err {worst:.2e}", flush=True)


def test_solve_P_c1(hsd, c1):
    w, ctx, gid, u = c1
    ud = torch.tensor(u[:16], device="cuda")
    Pd = torch.empty((16, 256), dtype=torch.float64, device="cuda")
    ctx.hsd_solve_P(ud, gid, Pd)
    ctx.hsd_sync()
    P = Pd.cpu().numpy()
    worst = 0.0
    for c in range(16):
        Pref, _ = oracle.solve_pair(u[c], w.grains[0], w.lam_cm)
        assert abs(P[c].sum() - 1.0) < 1e-13
        m = Pref >= 1e-6 * Pref.max()
        worst = max(worst, float(np.max(np.abs(P[c][m] / Pref[m] - 1))))
    print(f"c1 end-to-end worst P rel err (P >= 1e-6 max) {worst:.2e}", flush=True)
    assert worst < J_TOL


def test_zero_and_bad_fields(hsd, c1):
    w, ctx, gid, u = c1
    uu = u[:6].copy()
    uu[0] = 0.0
    uu[1, 17] = np.nan
    uu[2, 3] = -1.0
    ud = torch.tensor(uu, device="cuda")
    j = torch.empty((6, 1, w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((6, 1, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, [gid], j, diag)
    with pytest.raises(hsd.HsdError) as ei:
        ctx.hsd_sync()
    assert ei.value.status == -5
    flags = diag.cpu().numpy()[:, 0, 3].astype(int)
    assert flags[0] & 1 and not flags[0] & 4
    assert flags[1] & 4 and flags[2] & 4 and not flags[3] & 4
    # zero field: P = delta_i0 exactly, j = emission of the ground bin
    Pd = torch.empty((1, 256), dtype=torch.float64, device="cuda")
    ctx.hsd_solve_P(ud[:1], gid, Pd)
    ctx.hsd_sync()
    P = Pd.cpu().numpy()[0]
    assert P[0] == 1.0 and np.all(P[1:] == 0.0)
    s = oracle.grain_setup(w.grains[0], w.lam_cm)
    assert j_rel_err(j.cpu().numpy()[0, 0].astype(np.float64), s.cabs * s.planck[0]) < J_TOL
    # the bad values are read as zero: same as the oracle with those entries zeroed
    fixed = uu[1].copy(); fixed[17] = 0.0
    _, jr = oracle.solve_pair(fixed, w.grains[0], w.lam_cm)
    assert j_rel_err(j.cpu().numpy()[1, 0].astype(np.float64), jr) < J_TOL


def test_deterministic(hsd, c1):
    w, ctx, gid, u = c1
    ud = torch.tensor(u, device="cuda")
    outs = []
    for _ in range(2):
        j = torch.empty((w.n_cells, 2, w.n_lambda), dtype=torch.float32, device="cuda")
        ctx.hsd_solve(ud, [gid, gid], j)
        ctx.hsd_sync()
        outs.append(j.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0][:, 0], outs[0][:, 1])


def test_contraction_modes_agree(hsd):
    # the split-BF16 contraction (default) against the FP32 one on every pair
    # of a batched subset: each j within 3 2^-16 of the FP32 result (plus FP32
    # accumulation order), and a bad mode rejected
    w = synth.workload("c2_batched")
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in w.grains]
    n = 512
    ud = torch.tensor(make_fields(w.lam_cm, w.field_recipe, w.n_cells, cells=np.arange(n)), device="cuda")
    assert ctx.hsd_get_contract() == hsd.CONTRACT_BF16X3
    out = {}
    for mode in (hsd.CONTRACT_BF16X3, hsd.CONTRACT_FP32):
        ctx.hsd_set_contract(mode)
        j = torch.empty((n, len(ids), w.n_lambda), dtype=torch.float32, device="cuda")
        ctx.hsd_solve(ud, ids, j)
        ctx.hsd_sync()
        out[mode] = j.cpu().numpy().astype(np.float64)
    ctx.hsd_set_contract(hsd.CONTRACT_BF16X3)
    a, b = out[hsd.CONTRACT_BF16X3], out[hsd.CONTRACT_FP32]
    # the range the tolerances cover: values down to 1e-10 of the pair's
    # maximum (far below, products of FP32-subnormal size may round to 0)
    m = b >= 1e-10 * b.max(axis=-1, keepdims=True)
    rel = np.abs(a[m] / b[m] - 1)
    print(f"split BF16 vs FP32 contraction: median {np.median(rel):.2e} max {rel.max():.2e} "
          f"over {m.sum()} values", flush=True)
    assert rel.max() < 3 * 2.0 ** -16 + 2e-6
    with pytest.raises(hsd.HsdError):
        ctx.hsd_set_contract(2)


def test_c2_full_batch_sampled_pairs(hsd):
    # the full batched workload (16384 cells x 32 radii) in one call, as the
    # benchmark runs it; sampled pairs against the oracle
    w = synth.workload("c2_batched")
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in w.grains]
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells)
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((w.n_cells, len(ids), w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((w.n_cells, len(ids), 4), dtype=torch.float32, device="cuda")
    # the benchmark's launch: autotuned class configurations (from its cache)
    # and a plan replayed with phase timing and concurrent classes
    from paper_1311_4627_amd import autotune
    tuned = autotune.tune(ctx, ud, ids, cache_path=os.path.join(ROOT, "paper_1311_4627_amd", "tuned.json"))
    print(f"c2 launch configuration: {tuned['cfg']} (cached: {tuned['cached']})", flush=True)
    for c, cfg in enumerate(tuned["cfg"]):          # a concurrent plan launches ordinary grids
        ctx.hsd_set_class_cfg(c, **dict(cfg, persistent=0))
    plan = ctx.hsd_plan_create(ud, ids, j, diag, flags=hsd.PLAN_TIMING | hsd.PLAN_CONCURRENT)
    plan.hsd_plan_launch()
    torch.cuda.synchronize()
    ctx.hsd_sync()
    print("c2 solved on the GPU", flush=True)
    # the eager solve in the default configuration agrees (bit for bit unless
    # the wide layout was chosen, which reorders FP64 sums)
    for c in range(hsd.N_CLASSES):
        ctx.hsd_set_class_cfg(c, kg=2, wide=0, persistent=0)
    je = torch.empty_like(j)
    ctx.hsd_solve(ud, ids, je, None)
    ctx.hsd_sync()
    rel = ((je - j).abs() / j.abs().clamp_min(1e-30 * float(j.abs().max()))).max().item()
    print(f"c2 plan vs eager: max rel diff {rel:.2e}", flush=True)
    assert rel < 1e-5
    # the same batch with the FP32 contraction (eager), for the oracle comparison below
    ctx.hsd_set_contract(hsd.CONTRACT_FP32)
    try:
        ctx.hsd_solve(ud, ids, je, None)
        ctx.hsd_sync()
    finally:
        ctx.hsd_set_contract(hsd.CONTRACT_BF16X3)
    cells = [0, 2222, 4097, 9999, 16383]
    grains = [0, 3, 7, 11, 15, 19, 23, 27, 31]
    jj = j[cells].cpu().numpy().astype(np.float64)
    j32 = je[cells].cpu().numpy().astype(np.float64)
    del je
    dd = diag[cells].cpu().numpy().astype(np.float64)
    worst = worst32 = 0.0
    for gi in grains:
        for ci, c in enumerate(cells):
            P, jr, d = oracle.solve_pair(u[c], w.grains[gi], w.lam_cm, with_diag=True)
            e = j_rel_err(jj[ci, gi], jr)
            e32 = j_rel_err(j32[ci, gi], jr)
            print(f"c2 cell {c} grain {gi} (n={w.grains[gi].n_bins}): j rel err {e:.2e} (FP32 contraction "
                  f"{e32:.2e})", flush=True)
            worst = max(worst, e)
            worst32 = max(worst32, e32)
            assert e < J_TOL and e32 < J_TOL
            assert abs(dd[ci, gi, 0] / d["absorbed"] - 1) < 1e-6
            assert abs(dd[ci, gi, 1] / d["emitted"] - 1) < J_TOL
    # energy bookkeeping over the whole batch: finite everywhere; emitted vs
    # representable absorbed power within the discretisation error of the
    # point-evaluated heating rates on coarse bins (a few per cent for the
    # intermediate radii, see the oracle's energy-balance pins)
    dall = diag.cpu().numpy()
    assert np.all(np.isfinite(dall)) and np.all(dall[..., :3] > 0)
    ratio = dall[..., 1] / dall[..., 2]
    print(f"c2 emitted/A_rep over the batch: min {ratio.min():.4f} max {ratio.max():.4f}", flush=True)
    assert np.all(np.abs(ratio - 1.0) < 0.15)
    print(f"c2 worst sampled j rel err {worst:.2e} (FP32 contraction {worst32:.2e}) over "
          f"{len(cells) * len(grains)} pairs", flush=True)
    plan.close()


def test_tiny_grain_matches_dense_master_equation(hsd):
    lam = synth.wavelength_grid_cm(400)
    g = synth.make_grain("carbonaceous", 6.0e-8, lam, n_bins=16, E_range_erg=(0.05 * oracle.EV, 40.0 * oracle.EV))
    ctx = hsd.Context(lam)
    gid = ctx.add_grain(g)
    u = make_fields(lam, synth.FieldRecipe(9, (0.3, 300.0), 0.0, None), 3)
    Pd = torch.empty((3, 16), dtype=torch.float64, device="cuda")
    ctx.hsd_solve_P(torch.tensor(u, device="cuda"), gid, Pd)
    ctx.hsd_sync()
    P = Pd.cpu().numpy()
    s = oracle.grain_setup(g, lam)
    for c in range(3):
        Pdense = oracle.dense_steady_state(om.heating_matrix(u[c], s), s.cool)
        m = Pdense >= 1e-6 * Pdense.max()
        assert np.max(np.abs(P[c][m] / Pdense[m] - 1)) < J_TOL


def test_empty_batches_are_no_ops(hsd, c1):
    w, ctx, gid, u = c1
    u0 = torch.empty((0, w.n_lambda), dtype=torch.float64, device="cuda")
    j0 = torch.empty((0, 1, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(u0, [gid], j0, None)
    ud = torch.tensor(u[:2], device="cuda")
    jz = torch.empty((2, 0, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, [], jz, None)
    ctx.hsd_sync()


def test_maximum_sizes_match_oracle(hsd):
    # the largest grid and grain the library takes: 1024 wavelengths, 1024 bins
    lam = synth.wavelength_grid_cm(1024)
    g = synth.make_grain("carbonaceous", 3.5e-8, lam, n_bins=1024)
    ctx = hsd.Context(lam)
    gid = ctx.add_grain(g)
    rec = synth.FieldRecipe(seed=77, U_range=(0.1, 1e5), jitter=0.3, tau_V_range=None)
    u = make_fields(lam, rec, 5)
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((5, 1, 1024), dtype=torch.float32, device="cuda")
    diag = torch.empty((5, 1, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, [gid], j, diag)
    ctx.hsd_sync()
    jj = j.cpu().numpy()[:, 0].astype(np.float64)
    for c in (0, 2, 4):
        _, jr = oracle.solve_pair(u[c], g, lam)
        e = j_rel_err(jj[c], jr)
        print(f"max sizes cell {c}: j rel err {e:.2e}", flush=True)
        assert e < J_TOL


def test_wide_enthalpy_range_matches_oracle(hsd):
    # Enthalpy grids spanning ten decades (1e-6 .. 2e4 eV), so the rows' rate
    # factor c0 r^k, which the solver applies once per lane and step (Horner
    # sums in r^-P), ranges over as many; one grain with 528 bins (15.5 of the
    # 32 slots of its layout lie below row 0) and one with 1024.  Faint,
    # attenuated fields and bright ones: j and the representable absorbed
    # power against the oracle.
    lam = synth.wavelength_grid_cm(500)
    ev = oracle.EV
    grains = [synth.make_grain("carbonaceous", 8e-8, lam, n_bins=528, E_range_erg=(1e-6 * ev, 2e4 * ev)),
              synth.make_grain("silicate", 30e-8, lam, n_bins=1024, E_range_erg=(1e-6 * ev, 2e4 * ev))]
    ctx = hsd.Context(lam)
    gids = [ctx.add_grain(g) for g in grains]
    faint = make_fields(lam, synth.FieldRecipe(seed=91, U_range=(0.1, 1.0), jitter=0.0, tau_V_range=(5.0, 20.0)), 2)
    bright = make_fields(lam, synth.FieldRecipe(seed=92, U_range=(1e3, 1e5), jitter=0.3, tau_V_range=None), 2)
    u = np.concatenate([faint, bright])
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((4, 2, 500), dtype=torch.float32, device="cuda")
    diag = torch.empty((4, 2, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, gids, j, diag)
    ctx.hsd_sync()
    jj = j.cpu().numpy().astype(np.float64)
    dd = diag.cpu().numpy().astype(np.float64)
    for gi, g in enumerate(grains):
        for c in range(4):
            _, jr, d = oracle.solve_pair(u[c], g, lam, with_diag=True)
            e = j_rel_err(jj[c, gi], jr)
            ea = abs(dd[c, gi, 2] / d["A_rep"] - 1.0)
            print(f"wide E range: grain {gi} ({g.n_bins} bins) cell {c}: j rel err {e:.2e}, A_rep rel err {ea:.2e}",
                  flush=True)
            assert e < J_TOL
            assert ea < 1e-4


@pytest.mark.parametrize("wide", [0, 1])
def test_lane_layouts_match_oracle(hsd, wide):
    # Each bin-count class in both of its lane layouts (the alternate one where
    # the class has it), with bin counts that leave part of the layout empty:
    # 992, 304, 208, 128, 96 and 16 bins (in the 128-bin class, 96 bins leave
    # 32 positions below row 0: four slots of the 8-lane layout); faint
    # attenuated, moderate and bright fields.  j, emitted and representable
    # absorbed power against the oracle.
    lam = synth.wavelength_grid_cm(500)
    bins = [992, 304, 208, 128, 96, 16]
    radii = [3.5e-8, 12e-8, 25e-8, 60e-8, 120e-8, 400e-8]
    grains = [synth.make_grain("carbonaceous" if i % 2 == 0 else "silicate", a, lam, n_bins=n)
              for i, (a, n) in enumerate(zip(radii, bins))]
    ctx = hsd.Context(lam)
    gids = [ctx.add_grain(g) for g in grains]
    for c in range(hsd.N_CLASSES):
        ctx.hsd_set_class_cfg(c, kg=4 if wide else 2, wide=wide if c != 2 else 0, persistent=0)
    u = np.concatenate([
        make_fields(lam, synth.FieldRecipe(seed=93, U_range=(0.1, 1.0), jitter=0.0, tau_V_range=(5.0, 20.0)), 1),
        make_fields(lam, synth.FieldRecipe(seed=94, U_range=(1.0, 100.0), jitter=0.3, tau_V_range=None), 1),
        make_fields(lam, synth.FieldRecipe(seed=95, U_range=(1e3, 1e5), jitter=0.3, tau_V_range=None), 1)])
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((3, len(gids), 500), dtype=torch.float32, device="cuda")
    diag = torch.empty((3, len(gids), 4), dtype=torch.float32, device="cuda")
    print(f"lane layouts: wide {wide}, bins {bins}", flush=True)
    ctx.hsd_solve(ud, gids, j, diag)
    ctx.hsd_sync()
    jj = j.cpu().numpy().astype(np.float64)
    dd = diag.cpu().numpy().astype(np.float64)
    worst = 0.0
    for gi, g in enumerate(grains):
        for c in range(3):
            _, jr, d = oracle.solve_pair(u[c], g, lam, with_diag=True)
            e = j_rel_err(jj[c, gi], jr)
            worst = max(worst, e)
            assert e < J_TOL, (g.n_bins, c, e)
            assert abs(dd[c, gi, 1] / d["emitted"] - 1) < J_TOL
            assert abs(dd[c, gi, 2] / d["A_rep"] - 1) < J_TOL
    print(f"lane layouts (wide {wide}): worst j rel err {worst:.2e}", flush=True)
    ctx.close()


def test_size_convolution_matches_oracle(hsd):
    # four radii of the batched workload, three cells: the library's solve and
    # convolution against the oracle's spectra and its weighted sum
    w = synth.workload("c2_batched", n_cells=3)
    sel = [4, 12, 20, 31]
    grains = [w.grains[i] for i in sel]
    radii = synth.radii_cm(3.5, 250.0, 32)[sel]
    weights = synth.size_weights(radii)
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    u = make_fields(w.lam_cm, w.field_recipe, 16384, cells=np.array([0, 9000, 16383]))
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((3, 4, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, ids, j, None)
    out = torch.empty((3, w.n_lambda), dtype=torch.float64, device="cuda")
    ctx.hsd_size_convolve(j, weights, out)
    ctx.hsd_sync()
    got = out.cpu().numpy()
    # the weighted sum itself, on the library's own spectra
    mine = oracle.size_convolution(j.cpu().numpy(), weights, w.lam_cm)
    assert np.allclose(got, mine, rtol=1e-12, atol=0)
    for c in range(3):
        jr = np.stack([oracle.solve_pair(u[c], g, w.lam_cm)[1] for g in grains])
        ref = oracle.size_convolution(jr, weights, w.lam_cm)
        e = j_rel_err(got[c], ref)
        print(f"size convolution cell {c}: rel err {e:.2e}", flush=True)
        assert e < J_TOL
    # the paper's units: the same sums in eV (1 eV = 1.602176634e-12 erg), and
    # without the lambda weight
    out2 = torch.empty_like(out)
    ctx.hsd_size_convolve(j, weights, out2, per_ev=True)
    ctx.hsd_sync()
    assert np.allclose(out2.cpu().numpy(), mine / oracle.EV, rtol=1e-12, atol=0)
    ctx.hsd_size_convolve(j, weights, out2, lambda_weighted=False)
    ctx.hsd_sync()
    assert np.allclose(out2.cpu().numpy() * w.lam_cm[None, :], mine, rtol=1e-12, atol=0)
    # an unknown flag bit is refused (through the C ABI: the binding passes known bits only)
    w64 = np.ascontiguousarray(weights, dtype=np.float64)
    st = ctx._lib.hsd_size_convolve(ctx._h, 3, 4, j.data_ptr(), hsd._dptr(w64), 4, out2.data_ptr(), None)
    assert hsd.STATUS_NAMES.get(st) == "HSD_ERR_INVALID_ARG"
