"""The table method on the GPU (hsd_table_build / hsd_table_eval through the
C ABI) against its FP64 twin in the oracle (oracle/table.py): node spectra
per absorbed power to the plain path's 1e-4, and looked-up spectra to 1e-4
for cells inside, at the ends of and beyond the node range; the energy
budget of a table (the reference of the surrogate's table check) against its
twin."""

import math

import numpy as np
import pytest

import synth
from oracle import table as otab
from synth.fields import FieldRecipe, make_fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

J_TOL = 1e-4


def rel_err(j, jref):
    m = jref >= 1e-10 * jref.max()
    return float(np.max(np.abs(j[m] / jref[m] - 1.0))) if np.any(m) else 0.0


@pytest.fixture(scope="module")
def hsd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4627_amd import hsd as h
    return h


LO, HI, K = -1.0, 5.0, 13


@pytest.fixture(scope="module")
def twin():
    # four grains of the surrogate workload (1024, ~400, 128 bins; a silicate
    # grain), the unit reference field and the oracle's table of them
    w = synth.workload("c5_surrogate", n_cells=1)
    grains = [w.grains[i] for i in (0, 20, 63, 90)]
    u_ref = make_fields(w.lam_cm, FieldRecipe(0, (1.0, 1.0), 0.0, None), 1)[0]
    yo = [otab.build_table(g, w.lam_cm, u_ref, LO, HI, K) for g in grains]
    return w, grains, u_ref, yo


def test_table_matches_oracle_twin(hsd, twin):
    w, grains, u_ref, yo = twin
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    ur = torch.tensor(u_ref, device="cuda")
    lo, hi = LO, HI
    table = torch.empty((len(ids), K, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_table_build(ids, ur, lo, hi, table)
    ctx.hsd_sync()
    tg = table.cpu().numpy().astype(np.float64)
    worst = 0.0
    for gi in range(len(ids)):
        for k in range(K):
            jo = np.exp2(yo[gi][k])
            jg = np.where(tg[gi, k] > -1e29, np.exp2(tg[gi, k]), 0.0)
            worst = max(worst, rel_err(jg, jo))
    print(f"table nodes: worst rel err of j / A {worst:.2e}", flush=True)
    assert worst < J_TOL
    # cells of the surrogate workload's generator, plus three outside / at the ends of the range
    n = 12
    u = make_fields(w.lam_cm, w.field_recipe, 262144, cells=np.arange(0, 262144, 262144 // n)[:n])
    u = np.concatenate([u, [1e-3 * u_ref, 1e6 * u_ref, 10.0 ** lo * u_ref]])
    ud = torch.tensor(u, device="cuda")
    j = torch.empty((u.shape[0], len(ids), w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_table_eval(ud, ids, ur, lo, hi, table, j)
    ctx.hsd_sync()
    jj = j.cpu().numpy().astype(np.float64)
    worst = 0.0
    for c in range(u.shape[0]):
        for gi, g in enumerate(grains):
            ref = otab.lookup(yo[gi], lo, hi, u[c], u_ref, g.cabs_cm2, w.lam_cm)
            worst = max(worst, rel_err(jj[c, gi], ref))
    print(f"table lookups: worst rel err {worst:.2e} over {u.shape[0] * len(ids)} pairs", flush=True)
    assert worst < J_TOL
    with pytest.raises(hsd.HsdError):
        ctx.hsd_table_eval(ud, ids, ur, hi, lo, table, j)          # empty node range
    ctx.close()


def test_energy_budget_matches_oracle(hsd, twin):
    # the surrogate's table check takes as reference B = A rho(t): the oracle's
    # table (rounded to the storage's FP32) is the input, and the node ratios,
    # the cells' node coordinates and B are compared with the oracle's twin of
    # them (B is stored in FP32: 1e-5)
    from synth import surrogate as ssur
    w, grains, u_ref, yo = twin
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    G = len(ids)
    ur = torch.tensor(u_ref, device="cuda")
    y32 = np.stack([np.where(np.isfinite(y), y, -1.0e30) for y in yo]).astype(np.float32)
    yh = np.where(y32 > -1e29, y32.astype(np.float64), -np.inf)
    table = torch.tensor(y32, device="cuda")
    n = 12
    u = make_fields(w.lam_cm, w.field_recipe, 262144, cells=np.arange(0, 262144, 262144 // n)[:n])
    u = np.concatenate([u, [1e-3 * u_ref, 1e6 * u_ref, 10.0 ** LO * u_ref, 10.0 ** (0.5 * (LO + HI)) * u_ref]])
    ud = torch.tensor(u, device="cuda")
    # an untrained network whose statistics keep its spectra within a decade
    # or so of j / A = 1 (finite emitted power: a check that no pair fails)
    from oracle import mlp
    sur = hsd.Surrogate(ctx)
    sur.hsd_sur_set_params(ssur.init_params(ssur.n_outputs(w.n_lambda), seed=3))
    X = np.stack([mlp.features(uc, w.lam_cm, grains[0].radius_cm) for uc in u])
    sur.hsd_sur_set_norm(X.mean(axis=0), X.std(axis=0) + 1.0, np.zeros(sur.n_out), np.full(sur.n_out, 0.1))
    j = torch.empty((u.shape[0], G, w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((u.shape[0], G, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(hsd.HsdError):                            # no budget yet
        ctx.hsd_solve_surrogate(ud, ids, [sur] * G, j, diag, check=hsd.CHECK_TABLE)
    with pytest.raises(hsd.HsdError):                            # a grain twice
        ctx.hsd_set_energy_budget([ids[0], ids[0]], ur, LO, HI, table[:2])
    with pytest.raises(hsd.HsdError):                            # an empty node range
        ctx.hsd_set_energy_budget(ids, ur, HI, LO, table)
    with pytest.raises(hsd.HsdError):                            # a grain the context does not know
        ctx.hsd_set_energy_budget([ids[0], 999], ur, LO, HI, table[:2])
    ctx.hsd_set_energy_budget(ids[:2], ur, LO, HI, table[:2])
    with pytest.raises(hsd.HsdError):                            # grains 2, 3 have none
        ctx.hsd_solve_surrogate(ud, ids, [sur] * G, j, diag, check=hsd.CHECK_TABLE)
    ctx.hsd_set_energy_budget(ids, ur, LO, HI, table)
    # a tolerance no pair fails: every pair keeps the network's value and
    # carries its reference B
    nfb = ctx.hsd_solve_surrogate(ud, ids, [sur] * G, j, diag, tol=1e30, check=hsd.CHECK_TABLE)
    ctx.hsd_sync()
    assert nfb == 0
    dd = diag.cpu().numpy().astype(np.float64)
    worst = 0.0
    for gi, g in enumerate(grains):
        rho = otab.node_ratios(yh[gi], w.lam_cm)
        for c in range(u.shape[0]):
            A = otab.absorbed_power(u[c], g.cabs_cm2, w.lam_cm)
            B = A * otab.budget_ratio(rho, LO, HI, u[c], u_ref, w.lam_cm)
            worst = max(worst, abs(dd[c, gi, 2] / B - 1.0))
    print(f"table budget: worst rel err of B {worst:.2e} over {u.shape[0] * G} pairs", flush=True)
    assert worst < 1e-5
    # the 1% check: the pairs that fail it are the plain solve bit for bit
    je = torch.empty_like(j)
    de = torch.empty_like(diag)
    ctx.hsd_solve(ud, ids, je, de)
    nfb = ctx.hsd_solve_surrogate(ud, ids, [sur] * G, j, diag, tol=0.01, check=hsd.CHECK_TABLE)
    ctx.hsd_sync()
    dd = diag.cpu().numpy()
    surp = (dd[..., 3].astype(np.int32) & 8) != 0
    assert nfb == int(np.sum(~surp))
    assert np.all(np.abs(dd[surp][:, 1] / dd[surp][:, 2] - 1) <= 0.01 + 1e-6)
    fb = torch.tensor(~surp, device="cuda")
    assert torch.equal(j[fb], je[fb]) and torch.equal(diag[fb], de[fb])
    sur.close()
    ctx.close()
