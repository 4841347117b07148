"""The table method on the GPU (hsd_table_build / hsd_table_eval through the
C ABI) against its FP64 twin in the oracle (oracle/table.py): node spectra
per absorbed power to the plain path's 1e-4, and looked-up spectra to 1e-4
for cells inside, at the ends of and beyond the node range."""

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


def test_table_matches_oracle_twin(hsd):
    w = synth.workload("c5_surrogate", n_cells=1)
    sel = [0, 20, 63, 90]                          # 1024, ~400, 128 bins; a silicate grain
    grains = [w.grains[i] for i in sel]
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    u_ref = make_fields(w.lam_cm, FieldRecipe(0, (1.0, 1.0), 0.0, None), 1)[0]
    ur = torch.tensor(u_ref, device="cuda")
    lo, hi, K = -1.0, 5.0, 13
    table = torch.empty((len(ids), K, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_table_build(ids, ur, lo, hi, table)
    ctx.hsd_sync()
    tg = table.cpu().numpy().astype(np.float64)
    yo = [otab.build_table(g, w.lam_cm, u_ref, lo, hi, K) for g in grains]
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
