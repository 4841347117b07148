"""The learned surrogate on the GPU, through the C ABI, against the FP64
reference MLP (oracle/mlp.py), the plain solve and the FP64 oracle.

* features and targets: same values as the reference (FP32 storage);
* loss and gradient of the BF16 products: against the reference run with its
  matrix-product operands rounded to bfloat16 (the GPU accumulates in FP32,
  the reference in FP64, and an operand computed in FP32 may round to the
  other neighbour now and then), within 5e-3 of the gradient's norm;
* training: the loss falls, the held-out band error is small and far below
  that of an emissivity table indexed by the field strength alone (the cheap
  method the surrogate replaces);
* the fallback: pairs failing the 1% energy check are re-solved by the plain
  path bit for bit, the others pass the check (against the network's rho A,
  the absorbed power A, or a table's energy budget); tol = 0 reproduces the
  plain solve exactly.
"""

import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from synth import surrogate as ssur
from synth.fields import make_fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hsd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4627_amd import hsd as h
    return h


def _training_set(hsd, n_cells, composition="carbonaceous", heldout=False):
    # the first n_cells cells of the training (or held-out) stream
    w = synth.workload("c4_train")
    rec = w.notes["heldout_recipe"] if heldout else w.field_recipe
    n_total = w.notes["heldout_cells"] if heldout else w.n_cells
    grains = [g for g in w.grains if g.composition == composition]
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    u = make_fields(w.lam_cm, rec, n_total, cells=np.arange(n_cells))
    ud = torch.tensor(u, device="cuda")
    G = len(ids)
    j = torch.empty((n_cells, G, w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((n_cells, G, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(ud, ids, j, diag)
    X = torch.empty((n_cells * G, 33), dtype=torch.float32, device="cuda")
    A = torch.empty((n_cells * G,), dtype=torch.float64, device="cuda")
    ctx.hsd_sur_features(ud, ids, X, A)
    Y = torch.empty((n_cells * G, ssur.n_outputs(w.n_lambda)), dtype=torch.float32, device="cuda")
    ctx.hsd_sur_targets(j.view(-1, w.n_lambda), A, Y)
    ctx.hsd_sync()
    return dict(w=w, ctx=ctx, ids=ids, grains=grains, u=u, ud=ud, j=j, diag=diag, X=X, A=A, Y=Y)


@pytest.fixture(scope="module")
def small(hsd):
    return _training_set(hsd, 96)


def test_features_and_targets_match_reference(hsd, small):
    d = small
    w, G = d["w"], len(d["ids"])
    X = d["X"].cpu().numpy().reshape(-1, G, 33)
    A = d["A"].cpu().numpy().reshape(-1, G)
    Y = d["Y"].cpu().numpy().reshape(-1, G, ssur.n_outputs(w.n_lambda))
    j = d["j"].cpu().numpy()
    for c in (0, 37, 95):
        for g in (0, 21, 63):
            gr = d["grains"][g]
            xr = mlp.features(d["u"][c], w.lam_cm, gr.radius_cm)
            assert np.max(np.abs(X[c, g] - xr)) < 1e-5
            s = oracle.grain_setup(gr, w.lam_cm)
            Ar = float(np.trapezoid(oracle.C * d["u"][c] * s.cabs, w.lam_cm))
            assert abs(A[c, g] / Ar - 1) < 1e-12
            yr = mlp.targets(j[c, g].astype(np.float64), Ar, w.lam_cm)
            assert np.max(np.abs(Y[c, g] - yr)) < 1e-5


def test_features_do_not_depend_on_the_selection(hsd, small):
    # selections of 16 or fewer, 17..32 and more grains take differently
    # shaped blocks; every pair's inputs and absorbed power stay bit-identical
    d = small
    G = len(d["ids"])
    X = d["X"].cpu().numpy().reshape(-1, G, 33)
    A = d["A"].cpu().numpy().reshape(-1, G)
    n = X.shape[0]
    for cols in (list(range(16)), [3, 9, 40, 41, 63], list(range(20, 40)), list(range(0, 64, 2))):
        ids = [d["ids"][c] for c in cols]
        Xs = torch.empty((n * len(cols), 33), dtype=torch.float32, device="cuda")
        As = torch.empty((n * len(cols),), dtype=torch.float64, device="cuda")
        d["ctx"].hsd_sur_features(d["ud"], ids, Xs, As)
        d["ctx"].hsd_sync()
        print(f"selection of {len(cols)} grains", flush=True)
        assert np.array_equal(Xs.cpu().numpy().reshape(n, len(cols), 33), X[:, cols])
        assert np.array_equal(As.cpu().numpy().reshape(n, len(cols)), A[:, cols])


@pytest.mark.parametrize("band_weight", [0.0, 0.8])
def test_loss_and_gradient_match_bf16_reference(hsd, small, band_weight):
    d = small
    sur = hsd.Surrogate(d["ctx"])
    flat = ssur.init_params(ssur.n_outputs(d["w"].n_lambda), seed=99)
    sur.hsd_sur_set_params(flat)
    sur.hsd_sur_fit_norm(d["X"], d["Y"])
    sur.hsd_sur_set_loss(band_weight)
    xm, xs, ym, ys = sur.hsd_sur_get_norm()
    Xr, Yr = d["X"].cpu().numpy().astype(np.float64), d["Y"].cpu().numpy().astype(np.float64)
    mu, sd = mlp.zscore_stats(Xr)
    assert np.allclose(xm, mu, rtol=1e-5, atol=1e-5) and np.allclose(xs, sd, rtol=1e-4)
    mu, sd = mlp.target_stats(Yr)
    assert np.allclose(ym, mu, rtol=1e-5, atol=1e-5) and np.allclose(ys, sd, rtol=1e-4)
    n = 512
    rows = np.random.default_rng(3).choice(Xr.shape[0], n, replace=False)
    Xb = torch.tensor(Xr[rows], dtype=torch.float32, device="cuda")
    Yb = torch.tensor(Yr[rows], dtype=torch.float32, device="cuda")
    loss, g = sur.hsd_sur_loss_grad(Xb, Yb)
    # reference on the same normalised rows (the GPU's FP32 statistics)
    Xn = (Xr[rows] - xm) / xs
    Yn = (Yr[rows] - ym) / ys
    widths = ssur.widths(ssur.n_outputs(d["w"].n_lambda))
    Wt = mlp.loss_weights(Yr[rows], d["w"].lam_cm, band_weight)      # from the raw targets
    lref, gref = mlp.loss_and_grad(flat.astype(np.float64), widths, Xn, Yn, bf16=True, weights=Wt)
    print(f"loss {loss:.6e} ref {lref:.6e}", flush=True)
    assert abs(loss / lref - 1) < 1e-3
    # element by element: every gradient entry within 2^-8 of the sum of the
    # absolute values of its terms (an operand rounded to the other BF16
    # neighbour moves one term by at most 2^-7 of itself; FP32 accumulation of
    # K = 512 terms adds at most 512 2^-24 of that sum; an emulation with FP32
    # accumulation stays below 1.2e-3 of it; the device's FP32 loss weights
    # differ from the reference's by ~1e-6 relative)
    T = mlp.grad_abs_terms(flat.astype(np.float64), widths, Xn, Yn, weights=Wt)
    layers_g = mlp.unpack(g.astype(np.float64), widths)
    layers_r = mlp.unpack(gref, widths)
    layers_t = mlp.unpack(T, widths)
    for li, ((gw, gb), (rw, rb), (tw, tb)) in enumerate(zip(layers_g, layers_r, layers_t)):
        rw_ = np.abs(gw - rw) / tw
        rb_ = np.abs(gb - rb) / tb
        ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
        print(f"layer {li}: dW max |g - g_ref| / sum|terms| {rw_.max():.2e} (norm rel {ew:.2e}), "
              f"db {rb_.max():.2e}; median |g_ref| / sum|terms| {np.median(np.abs(rw) / tw):.2e}", flush=True)
        assert rw_.max() <= 2.0 ** -8 and rb_.max() <= 2.0 ** -8
    sur.close()


def test_training_lowers_loss_and_beats_a_table(hsd):
    d = _training_set(hsd, 4096)
    h = _training_set(hsd, 64, heldout=True)
    w, G = d["w"], len(d["ids"])
    sur = hsd.Surrogate(d["ctx"])
    sur.hsd_sur_set_params(ssur.init_params(ssur.n_outputs(w.n_lambda)))
    sur.hsd_sur_fit_norm(d["X"], d["Y"])
    trace = sur.hsd_sur_train(d["X"], d["Y"], steps=4000, batch=4096, lr=4e-3)
    print(f"loss: first {trace[:20].mean():.4e} last {trace[-50:].mean():.4e}", flush=True)
    assert np.all(np.isfinite(trace)) and trace[-50:].mean() < 0.05 * trace[:20].mean()
    # held-out pairs through the trained network (same context as the training grains)
    hu = torch.tensor(h["u"], device="cuda")
    jp = torch.empty_like(h["j"])
    dp = torch.empty_like(h["diag"])
    sur.hsd_sur_predict(hu, d["ids"], jp, dp)
    torch.cuda.synchronize()
    jp = jp.cpu().numpy().reshape(-1, w.n_lambda)
    jr = h["j"].cpu().numpy().reshape(-1, w.n_lambda)
    err_net = mlp.band_rel_error(jp, jr, w.lam_cm)
    # the table method: the training pair of the same grain with the nearest
    # total field energy, its spectrum per absorbed power times this pair's A
    Xt = d["X"].cpu().numpy().reshape(-1, G, 33)
    Yt = d["Y"].cpu().numpy().reshape(-1, G, ssur.n_outputs(w.n_lambda))[..., :w.n_lambda]
    Xh = h["X"].cpu().numpy().reshape(-1, G, 33)
    Ah = h["A"].cpu().numpy().reshape(-1, G)
    etot_t = np.log10(np.sum(10.0 ** Xt[:, 0, :32].astype(np.float64), axis=1))
    etot_h = np.log10(np.sum(10.0 ** Xh[:, 0, :32].astype(np.float64), axis=1))
    nn = np.argmin(np.abs(etot_h[:, None] - etot_t[None, :]), axis=1)
    jt = (10.0 ** Yt[nn].astype(np.float64)) * Ah[..., None]
    err_tab = mlp.band_rel_error(jt.reshape(-1, w.n_lambda), jr, w.lam_cm)
    print(f"held-out band error: network median {np.median(err_net):.4f} p99 {np.quantile(err_net, 0.99):.4f} "
          f"max {err_net.max():.4f}; table median {np.median(err_tab):.4f} max {err_tab.max():.4f}", flush=True)
    assert np.median(err_net) < 0.5 * np.median(err_tab)
    assert np.median(err_net) < 0.05
    sur.close()


def test_fallback_is_the_plain_solve(hsd, small):
    d = small
    w, ctx, ids = d["w"], d["ctx"], d["ids"]
    sur = hsd.Surrogate(ctx)
    sur.hsd_sur_set_params(ssur.init_params(ssur.n_outputs(w.n_lambda), seed=5))
    sur.hsd_sur_fit_norm(d["X"], d["Y"])
    sur.hsd_sur_train(d["X"], d["Y"], steps=400, batch=512, lr=2e-3)
    G = len(ids)
    n_cells = d["u"].shape[0]
    j = torch.empty((n_cells, G, w.n_lambda), dtype=torch.float32, device="cuda")
    diag = torch.empty((n_cells, G, 4), dtype=torch.float32, device="cuda")
    jp = torch.empty_like(j)
    dp = torch.empty_like(diag)
    sur.hsd_sur_predict(d["ud"], ids, jp, dp)
    nfb = ctx.hsd_solve_surrogate(d["ud"], ids, [sur] * G, j, diag, tol=0.01)
    ctx.hsd_sync()
    flags = diag[..., 3].to(torch.int32).cpu().numpy()
    surp = (flags & 8) != 0
    print(f"fallback {nfb} of {n_cells * G} pairs", flush=True)
    assert nfb == int(np.sum(~surp))
    pflags = dp[..., 3].to(torch.int32).cpu().numpy()
    assert np.array_equal(~surp, (pflags & 16) != 0)
    # surrogate pairs: the prediction, and the energy check holds against the
    # model's predicted budget rho A (diag entry 2)
    assert torch.equal(j[torch.tensor(surp, device="cuda")], jp[torch.tensor(surp, device="cuda")])
    dd = diag.cpu().numpy()
    assert np.all(np.abs(dd[surp][:, 1] / dd[surp][:, 2] - 1) <= 0.01 + 1e-6)
    assert np.array_equal(dd[surp][:, 2], dp.cpu().numpy()[surp][:, 2])
    # fallback pairs: exactly the plain solve
    je, de = d["j"], d["diag"]
    fb = torch.tensor(~surp, device="cuda")
    assert torch.equal(j[fb], je[fb]) and torch.equal(diag[fb], de[fb])
    # the check against the absorbed power itself
    nfa = ctx.hsd_solve_surrogate(d["ud"], ids, [sur] * G, j, diag, tol=0.01, check=hsd.CHECK_ABSORBED)
    ctx.hsd_sync()
    dd = diag.cpu().numpy()
    surp = (dd[..., 3].astype(np.int32) & 8) != 0
    print(f"fallback (check against A) {nfa} of {n_cells * G} pairs", flush=True)
    assert nfa == int(np.sum(~surp))
    assert np.all(np.abs(dd[surp][:, 1] / dd[surp][:, 0] - 1) <= 0.01 + 1e-6)
    assert np.array_equal(dd[surp][:, 2], dd[surp][:, 0])
    fb = torch.tensor(~surp, device="cuda")
    assert torch.equal(j[fb], je[fb]) and torch.equal(diag[fb], de[fb])
    # the check against a table's energy budget (the table built by the plain
    # path for these grains): B in diag entry 2, the same fallback rule
    from synth.fields import FieldRecipe
    u_ref = torch.tensor(make_fields(w.lam_cm, FieldRecipe(0, (1.0, 1.0), 0.0, None), 1)[0], device="cuda")
    table = torch.empty((G, 25, w.n_lambda), dtype=torch.float32, device="cuda")
    ctx.hsd_table_build(ids, u_ref, -2.0, 6.0, table)
    ctx.hsd_set_energy_budget(ids, u_ref, -2.0, 6.0, table)
    del table
    nft = ctx.hsd_solve_surrogate(d["ud"], ids, [sur] * G, j, diag, tol=0.01, check=hsd.CHECK_TABLE)
    ctx.hsd_sync()
    dd = diag.cpu().numpy()
    surp = (dd[..., 3].astype(np.int32) & 8) != 0
    print(f"fallback (check against the table budget) {nft} of {n_cells * G} pairs", flush=True)
    assert nft == int(np.sum(~surp))
    assert np.all(np.abs(dd[surp][:, 1] / dd[surp][:, 2] - 1) <= 0.01 + 1e-6)
    assert np.all(np.isfinite(dd[surp][:, 2])) and np.all(dd[surp][:, 2] > 0)
    fb = torch.tensor(~surp, device="cuda")
    assert torch.equal(j[fb], je[fb]) and torch.equal(diag[fb], de[fb])
    # tol = 0: every pair falls back and the output is the plain solve
    nfb0 = ctx.hsd_solve_surrogate(d["ud"], ids, [sur] * G, j, diag, tol=0.0)
    ctx.hsd_sync()
    assert nfb0 == n_cells * G
    assert torch.equal(j, je) and torch.equal(diag, de)
    with pytest.raises(hsd.HsdError):
        ctx.hsd_solve_surrogate(d["ud"], ids, [sur] * G, j, diag, tol=0.01, check=7)
    sur.close()


def test_inference_matches_bf16_reference(hsd, small):
    # the inference kernels (BF16 activations between weight-stationary
    # layers, spectrum epilogue) against the reference forward pass with
    # BF16-rounded operands, on the same raw inputs and statistics
    d = small
    w, G = d["w"], len(d["ids"])
    sur = hsd.Surrogate(d["ctx"])
    flat = ssur.init_params(ssur.n_outputs(w.n_lambda), seed=17)
    sur.hsd_sur_set_params(flat)
    sur.hsd_sur_fit_norm(d["X"], d["Y"])
    sur.hsd_sur_train(d["X"], d["Y"], steps=200, batch=512, lr=2e-3)     # weights away from their init
    flat = sur.hsd_sur_get_params().astype(np.float64)
    xm, xs, ym, ys = sur.hsd_sur_get_norm()
    n_cells = 24
    jp = torch.empty((n_cells, G, w.n_lambda), dtype=torch.float32, device="cuda")
    dp = torch.empty((n_cells, G, 4), dtype=torch.float32, device="cuda")
    sur.hsd_sur_predict(d["ud"][:n_cells].contiguous(), d["ids"], jp, dp)
    torch.cuda.synchronize()
    X = d["X"].cpu().numpy()[: n_cells * G].astype(np.float64)
    A = d["A"].cpu().numpy()[: n_cells * G]
    widths = ssur.widths(ssur.n_outputs(w.n_lambda))
    yhat, _ = mlp.forward(flat, widths, (X - xm) / xs, bf16=True)
    yraw = yhat * ys + ym
    jref = A[:, None] * 10.0 ** yraw[:, :w.n_lambda]
    jg = jp.cpu().numpy().reshape(-1, w.n_lambda).astype(np.float64)
    rel = np.abs(jg / jref - 1)
    # per element: the normalised output within 2^-8 of the sum of the
    # absolute values of its last-layer terms (the rounding bound of the
    # gradient test; an FP32-accumulation emulation stays below 7.6e-4 of it),
    # carried through j = A 10^(y sigma + mu), plus the FP32 exponential's
    # own rounding (1e-5)
    Yabs = mlp.output_abs_terms(flat, widths, (X - xm) / xs)
    bound = np.expm1(math.log(10.0) * ys[None, :w.n_lambda] * 2.0 ** -8 * Yabs[:, :w.n_lambda]) + 1e-5
    print(f"inference vs reference: median {np.median(rel):.2e} max {rel.max():.2e}; "
          f"max rel err / bound {np.max(rel / bound):.2e}", flush=True)
    assert np.all(rel <= bound)
    assert np.median(rel) < 2e-4
    # emitted power of each pair: 4 pi trapezoid of its spectrum
    em = 4 * math.pi * np.trapezoid(jg, w.lam_cm, axis=1)
    dg = dp.cpu().numpy().reshape(-1, 4).astype(np.float64)
    assert np.allclose(dg[:, 1], em, rtol=1e-5)
    # the energy-ratio output: diag entry 2 = rho A
    rho = dg[:, 2] / dg[:, 0]
    rr = np.abs(rho / 10.0 ** yraw[:, w.n_lambda] - 1)
    rbound = np.expm1(math.log(10.0) * ys[w.n_lambda] * 2.0 ** -8 * Yabs[:, w.n_lambda]) + 1e-5
    print(f"energy ratio vs reference: max {rr.max():.2e}, max / bound {np.max(rr / rbound):.2e}", flush=True)
    assert np.all(rr <= rbound)
    sur.close()


def test_fallback_beyond_the_flag_list(hsd):
    # more flagged pairs than the check's list holds (2^20): the fallback
    # scans every pair's flags instead, and tol = 0 still gives the plain solve
    w = synth.workload("c4_train")
    grains = [g for g in w.grains if g.composition == "carbonaceous"]
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in grains]
    n_cells = 16448                      # 16448 x 64 = 1,052,672 pairs > 2^20
    u = torch.tensor(make_fields(w.lam_cm, w.field_recipe, n_cells), device="cuda")
    G, L = len(ids), w.n_lambda
    je = torch.empty((n_cells, G, L), dtype=torch.float32, device="cuda")
    de = torch.empty((n_cells, G, 4), dtype=torch.float32, device="cuda")
    ctx.hsd_solve(u, ids, je, de)
    sur = hsd.Surrogate(ctx)
    sur.hsd_sur_set_params(ssur.init_params(ssur.n_outputs(L), seed=23))
    sur.hsd_sur_set_norm(np.full(33, -3.0), np.full(33, 2.0), np.full(L + 1, -2.0), np.full(L + 1, 0.5))
    j = torch.empty_like(je)
    d = torch.empty_like(de)
    nfb = ctx.hsd_solve_surrogate(u, ids, [sur] * G, j, d, tol=0.0)
    ctx.hsd_sync()
    print(f"fallback {nfb} of {n_cells * G} pairs", flush=True)
    assert nfb == n_cells * G
    assert torch.equal(j, je) and torch.equal(d, de)
    sur.close()


def test_training_is_deterministic_and_resumes_from_a_checkpoint(hsd, small, tmp_path):
    # two networks trained from the same initial weights, statistics and seed
    # hold the same bits; a network loaded from a checkpoint taken after N
    # steps and trained M more equals the saved network trained M more
    d = small
    w = d["w"]
    flat = ssur.init_params(ssur.n_outputs(w.n_lambda), seed=31)
    nets = []
    for _ in range(2):
        sur = hsd.Surrogate(d["ctx"])
        sur.hsd_sur_set_params(flat)
        sur.hsd_sur_fit_norm(d["X"], d["Y"])
        nets.append(sur)
    stats = [s.hsd_sur_get_norm() for s in nets]
    for a, b in zip(*stats):
        assert np.array_equal(a, b)
    t0 = nets[0].hsd_sur_train(d["X"], d["Y"], steps=120, batch=512, lr=2e-3, seed=11)
    t1 = nets[1].hsd_sur_train(d["X"], d["Y"], steps=120, batch=512, lr=2e-3, seed=11)
    assert np.array_equal(t0, t1)
    assert np.array_equal(nets[0].hsd_sur_get_params(), nets[1].hsd_sur_get_params())
    print("same seed: identical weights and loss traces", flush=True)
    # training steps replayed from one captured graph (the default) give the
    # bits of eager launches, also over two calls with other work between them
    def fresh_net(graph):
        sur = hsd.Surrogate(d["ctx"])
        sur.hsd_sur_set_params(flat)
        sur.hsd_sur_fit_norm(d["X"], d["Y"])
        sur.hsd_sur_set_train_graph(graph)
        return sur
    eager = fresh_net(False)
    te = eager.hsd_sur_train(d["X"], d["Y"], steps=120, batch=512, lr=2e-3, seed=11)
    assert np.array_equal(te, t0)
    assert np.array_equal(eager.hsd_sur_get_params(), nets[0].hsd_sur_get_params())
    g2, e2 = fresh_net(True), fresh_net(False)
    jx = torch.empty((8, len(d["ids"]), w.n_lambda), dtype=torch.float32, device="cuda")
    ga = g2.hsd_sur_train(d["X"], d["Y"], steps=60, batch=512, lr=2e-3, seed=11)
    g2.hsd_sur_predict(d["ud"][:8].contiguous(), d["ids"], jx)
    torch.cuda.synchronize()
    gb = g2.hsd_sur_train(d["X"], d["Y"], steps=60, batch=512, lr=2e-3, seed=11)
    ea = e2.hsd_sur_train(d["X"], d["Y"], steps=60, batch=512, lr=2e-3, seed=11)
    eb = e2.hsd_sur_train(d["X"], d["Y"], steps=60, batch=512, lr=2e-3, seed=11)
    assert np.array_equal(ga, ea) and np.array_equal(gb, eb)
    assert np.array_equal(g2.hsd_sur_get_params(), e2.hsd_sur_get_params())
    print("graph-replayed and eager training: identical weights and loss traces", flush=True)
    # checkpoint after N = 120 steps, then M = 80 more on both sides
    path = str(tmp_path / "net.hsdsur")
    nets[1].hsd_surrogate_save(path)
    resumed = hsd.Surrogate(d["ctx"])
    resumed.hsd_surrogate_load(path)
    assert np.array_equal(resumed.hsd_sur_get_params(), nets[1].hsd_sur_get_params())
    for a, b in zip(resumed.hsd_sur_get_norm(), nets[1].hsd_sur_get_norm()):
        assert np.array_equal(a, b)
    ta = nets[1].hsd_sur_train(d["X"], d["Y"], steps=80, batch=512, lr=2e-3, seed=11)
    tb = resumed.hsd_sur_train(d["X"], d["Y"], steps=80, batch=512, lr=2e-3, seed=11)
    assert np.array_equal(ta, tb)
    assert np.array_equal(nets[1].hsd_sur_get_params(), resumed.hsd_sur_get_params())
    # without the optimiser state the continuation differs (the moments matter)
    wpath = str(tmp_path / "net_weights.hsdsur")
    nets[0].hsd_surrogate_save(wpath, weights_only=True)
    assert os.path.getsize(wpath) < 0.4 * os.path.getsize(path)
    fresh = hsd.Surrogate(d["ctx"])
    fresh.hsd_surrogate_load(wpath)
    assert np.array_equal(fresh.hsd_sur_get_params(), nets[0].hsd_sur_get_params())
    tc = fresh.hsd_sur_train(d["X"], d["Y"], steps=80, batch=512, lr=2e-3, seed=11)
    assert not np.array_equal(tc, ta)
    # weights-only checkpoints predict exactly what the saved network predicts
    n_cells, G = 8, len(d["ids"])
    ja = torch.empty((n_cells, G, w.n_lambda), dtype=torch.float32, device="cuda")
    jb = torch.empty_like(ja)
    nets[1].hsd_surrogate_save(wpath, weights_only=True)
    fresh.hsd_surrogate_load(wpath)
    nets[1].hsd_sur_predict(d["ud"][:n_cells].contiguous(), d["ids"], ja)
    fresh.hsd_sur_predict(d["ud"][:n_cells].contiguous(), d["ids"], jb)
    torch.cuda.synchronize()
    assert torch.equal(ja, jb)
    # files of another shape or a truncated file are rejected
    with open(path, "rb") as f:
        blob = f.read()
    bad = str(tmp_path / "bad.hsdsur")
    with open(bad, "wb") as f:
        f.write(blob[:-4])
    with pytest.raises(hsd.HsdError):
        fresh.hsd_surrogate_load(bad)
    with open(bad, "wb") as f:
        f.write(blob.replace(b'"n_params": ', b'"n_params": 1', 1))
    with pytest.raises(hsd.HsdError):
        fresh.hsd_surrogate_load(bad)
    for s in nets + [resumed, fresh]:
        s.close()
