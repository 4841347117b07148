"""Pins of the FP64 surrogate reference (oracle/mlp.py) against closed forms,
finite differences and independent library routines."""

import math

import numpy as np
import pytest
from scipy import integrate, stats

import synth
from oracle import mlp
from synth.fields import FieldRecipe, make_fields
from synth import surrogate as ssur

SMALL = (5, 7, 6, 3)


def _small_problem(seed=3):
    rng = np.random.default_rng(seed)
    n_p = sum(SMALL[i + 1] * SMALL[i] + SMALL[i + 1] for i in range(len(SMALL) - 1))
    flat = rng.normal(0.0, 0.7, n_p)
    X = rng.normal(0.0, 1.0, (9, SMALL[0]))
    Y = rng.normal(0.0, 1.0, (9, SMALL[-1]))
    return flat, X, Y


def test_gelu_matches_normal_cdf_definition_and_derivative():
    z = np.linspace(-6.0, 6.0, 241)
    assert np.allclose(mlp.gelu(z), z * stats.norm.cdf(z), rtol=1e-14, atol=1e-300)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(mlp.gelu(-z), mlp.gelu(z) - z, atol=1e-14)       # z Phi(-z) = z - z Phi(z)


def test_loss_gradient_against_central_differences():
    flat, X, Y = _small_problem()
    loss, g = mlp.loss_and_grad(flat, SMALL, X, Y)
    h = 1e-6
    fd = np.empty_like(flat)
    for k in range(flat.shape[0]):
        e = np.zeros_like(flat)
        e[k] = h
        fd[k] = (mlp.loss_and_grad(flat + e, SMALL, X, Y)[0] - mlp.loss_and_grad(flat - e, SMALL, X, Y)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))
    # the loss itself is the mean squared residual of the forward pass
    yhat, _ = mlp.forward(flat, SMALL, X)
    assert loss == pytest.approx(np.mean((yhat - Y) ** 2), rel=1e-15)


def test_full_size_gradient_spot_check():
    w = ssur.widths(500)
    flat = ssur.init_params(500, seed=11).astype(np.float64)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(6, 33))
    Y = rng.normal(size=(6, 500))
    _, g = mlp.loss_and_grad(flat, w, X, Y)
    h = 1e-5
    for k in rng.choice(flat.shape[0], 12, replace=False):
        e = np.zeros_like(flat)
        e[k] = h
        fd = (mlp.loss_and_grad(flat + e, w, X, Y)[0] - mlp.loss_and_grad(flat - e, w, X, Y)[0]) / (2 * h)
        assert abs(g[k] - fd) < 1e-7 * max(1e-3, abs(fd))


def test_pack_unpack_layout_and_parameter_count():
    w = ssur.widths(500)
    assert ssur.n_params(500) == 268788
    flat = ssur.init_params(500)
    layers = mlp.unpack(flat, w)
    assert [l[0].shape for l in layers] == [(256, 33), (256, 256), (256, 256), (500, 256)]
    assert np.array_equal(mlp.pack(layers), flat.astype(np.float64))
    # W1 is the first block, row-major [out][in]
    assert layers[0][0][1, 0] == flat[33]


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(0, 1, 5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)
    assert mlp.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0                  # tie to even
    assert mlp.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6    # tie to even, upward


def test_split_operand_keeps_sixteen_bits():
    # hi + lo reproduces the FP32 operand to about 2^-17 relative, so the split
    # product sits ~2^8 closer to the exact one than a single-term product
    # with the same bfloat16 weights
    rng = np.random.default_rng(11)
    a = rng.normal(0, 1.5, (400, 33))
    W = rng.normal(0, 0.3, (33, 64))
    hi = mlp.bf16_round(a)
    lo = mlp.bf16_round(np.asarray(a, np.float32) - hi.astype(np.float32))
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(hi))
    assert np.max(np.abs(hi + lo - a) / np.abs(a)) < 2.0 ** -16
    Wq = mlp.bf16_round(W)
    exact = a @ Wq
    e1 = np.abs(mlp._mm(a, W, True) - exact).max()
    e2 = np.abs(mlp._mm(a, W, True, split=True) - exact).max()
    assert e2 < e1 / 64
    assert np.array_equal(mlp._mm(a, W, False), a @ W)


def test_bf16_mode_is_close_to_fp64():
    flat, X, Y = _small_problem(9)
    l64, g64 = mlp.loss_and_grad(flat, SMALL, X, Y)
    l16, g16 = mlp.loss_and_grad(flat, SMALL, X, Y, bf16=True)
    assert abs(l16 / l64 - 1) < 2e-2
    assert np.linalg.norm(g16 - g64) < 2e-2 * np.linalg.norm(g64)


def test_adam_first_step_and_quadratic():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    # first step: bias-corrected m = g, v = g^2, so the move is lr * sign(g)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)
    # minimises a quadratic
    x = np.array([3.0, -4.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 3001):
        x, m, v = mlp.adam_step(x, 2.0 * x, m, v, t, 0.05)
    assert np.max(np.abs(x)) < 1e-2


def test_band_integrals_partition_the_grid_and_features():
    lam = synth.wavelength_grid_cm(500)
    e = mlp.band_edges(500)
    assert e[0] == 0 and e[-1] == 499 and np.all(np.diff(e) > 0)
    u = make_fields(lam, FieldRecipe(2, (0.1, 1e3), 0.0, None), 4)
    B = mlp.band_integrals(u, lam)
    assert np.allclose(B.sum(axis=-1), np.trapezoid(u, lam, axis=-1), rtol=1e-12)
    # one band against scipy's trapezoid on its own nodes
    assert B[1, 5] == pytest.approx(integrate.trapezoid(u[1, e[5]:e[6] + 1], lam[e[5]:e[6] + 1]), rel=1e-12)
    x = mlp.features(u, lam, 1e-7)
    assert x.shape == (4, 33) and np.all(x[:, 32] == -7.0)
    assert np.allclose(10 ** x[:, :32], B, rtol=1e-12)


def test_targets_and_band_error():
    lam = synth.wavelength_grid_cm(500)
    rng = np.random.default_rng(1)
    j = np.exp(rng.normal(size=(3, 500)))
    A = np.array([2.0, 3.0, 4.0])
    y = mlp.targets(j, A, lam)
    assert y.shape == (3, 501)
    assert np.allclose(10 ** y[:, :500] * A[:, None], j, rtol=1e-12)
    jz = j.copy()
    jz[0, :10] = 0.0
    assert np.all(np.isfinite(mlp.targets(jz, A, lam)))
    # the ratio column: for a spectrum linear in lambda the trapezoid rule is
    # exact, E = 4 pi (a (l1 - l0) + b (l1^2 - l0^2) / 2)
    a, b = 3.0, 5.0e4
    jl = a + b * lam
    E = 4.0 * np.pi * (a * (lam[-1] - lam[0]) + 0.5 * b * (lam[-1] ** 2 - lam[0] ** 2))
    yl = mlp.targets(jl[None, :], np.array([7.0]), lam)
    assert abs(10 ** yl[0, 500] * 7.0 / E - 1) < 1e-12
    assert np.all(mlp.band_rel_error(j, j, lam) == 0.0)
    assert np.allclose(mlp.band_rel_error(1.01 * j, j, lam), 0.01, rtol=1e-10)


def test_zscore_stats():
    A = np.array([[1.0, 5.0], [3.0, 5.0]])
    mu, sd = mlp.zscore_stats(A)
    assert np.allclose(mu, [2.0, 5.0]) and np.allclose(sd, [1.0, 1.0])
    # targets: spectrum columns share sqrt(mean variance), the ratio keeps its own
    Y = np.array([[0.0, 0.0, 1.0], [2.0, 4.0, 1.5]])
    mu, sd = mlp.target_stats(Y)
    assert np.allclose(mu, [1.0, 2.0, 1.25])
    assert np.allclose(sd, [np.sqrt((1.0 + 4.0) / 2)] * 2 + [0.25 * mlp.RATIO_SCALE])


def test_absolute_term_sums_by_brute_force():
    # the error scales the GPU parity bounds use: sums of |term| of every
    # gradient element and of every output, by explicit loops on a tiny net
    flat, X, Y = _small_problem(seed=8)
    T = mlp.grad_abs_terms(flat, SMALL, X, Y)
    _, g = mlp.loss_and_grad(flat, SMALL, X, Y, bf16=True)
    assert np.all(np.abs(g) <= T * (1 + 1e-12))               # triangle inequality
    layers = mlp.unpack(flat, SMALL)
    yhat, (hs, zs) = mlp.forward(flat, SMALL, X, bf16=True)
    n, m = yhat.shape
    dz = 2.0 * (yhat - Y) / (n * m)
    ref = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        n_out, n_in = W.shape
        tw = np.zeros((n_out, n_in))
        tb = np.zeros(n_out)
        for o in range(n_out):
            for k in range(n_in):
                for s in range(n):
                    tw[o, k] += abs(mlp.bf16_round(dz[s, o])) * abs(mlp.bf16_round(hs[i][s, k]))
            for s in range(n):
                tb[o] += abs(dz[s, o])
        ref.insert(0, (tw, tb))
        if i > 0:
            nz = np.zeros((n, n_in))
            for s in range(n):
                for k in range(n_in):
                    acc = 0.0
                    for o in range(n_out):
                        acc += mlp.bf16_round(dz[s, o]) * mlp.bf16_round(W[o, k])
                    nz[s, k] = acc * mlp.gelu_grad(zs[i - 1][s, k])
            dz = nz
    assert np.allclose(T, mlp.pack(ref), rtol=1e-12, atol=0)
    # outputs: last layer with its input split into hi and lo terms
    Yabs = mlp.output_abs_terms(flat, SMALL, X)
    assert np.all(np.abs(yhat) <= Yabs * (1 + 1e-12))
    W, b = layers[-1]
    for s in range(n):
        for o in range(W.shape[0]):
            acc = abs(b[o])
            for k in range(W.shape[1]):
                x = hs[-2][s, k]
                hi = mlp.bf16_round(x)
                lo = mlp.bf16_round(np.float32(x) - np.float32(hi))
                acc += (abs(hi) + abs(lo)) * abs(mlp.bf16_round(W[o, k]))
            assert Yabs[s, o] == pytest.approx(acc, rel=1e-12)


def test_band_loss_weights():
    # weights of the band-weighted loss: every row's spectrum weights average
    # to 1, the ratio output keeps 1, band_weight 0 is the plain loss; the
    # band error they target is first-order in the weighted log errors; and the
    # node weights integrate like the band integrals
    lam = synth.wavelength_grid_cm(500)
    q = mlp.band_node_weights(lam)
    rng = np.random.default_rng(12)
    f = rng.random((3, 500))
    assert np.allclose(f @ q.T, mlp.band_integrals(f, lam), rtol=1e-13)
    assert np.allclose(q.sum(axis=0)[1:-1] * 2, (lam[2:] - lam[:-2]), rtol=1e-13)
    # a smooth spectrum-like target: a blackbody-ish bump per row
    x = np.log(lam / 1e-3)
    Y = np.concatenate([(-3.0 * (x[None, :] - rng.normal(0, 1, (4, 1))) ** 2 / 4.0) / np.log(10) - 10.0,
                        rng.normal(0, 0.01, (4, 1))], axis=1)
    W0 = mlp.loss_weights(Y, lam, 0.0)
    assert np.all(W0 == 1.0)
    W = mlp.loss_weights(Y, lam, 0.9)
    assert np.all(W[:, -1] == 1.0) and np.all(W > 0)
    assert np.allclose(W[:, :-1].mean(axis=1), 1.0, rtol=1e-12)
    # first order: a small log error d changes each band by
    # ln10 sum_k d_k j_k q_kb / J_b, the sensitivity the weights are built from
    j = 10.0 ** Y[:, :-1]
    J = j @ q.T
    d = 1e-6 * rng.normal(size=j.shape)
    J2 = (10.0 ** (Y[:, :-1] + d)) @ q.T
    on = J >= 1e-3 * J.sum(axis=1, keepdims=True)
    pred = math.log(10) * (d * j) @ q.T / J
    assert np.allclose((J2 / J - 1)[on], pred[on], rtol=1e-4, atol=1e-11)
    # rho concentrates on the bands with power: zero weight share outside them
    rho = (W[:, :-1] - 0.1) / (0.9 * 500)
    dead = (q[~on[0]].sum(axis=0) > 0) & (q[on[0]].sum(axis=0) == 0)
    assert np.allclose(rho[0][dead], 0.0, atol=1e-15)
    assert abs(rho[0].sum() - 1.0) < 1e-12


def test_weighted_loss_gradient_against_central_differences():
    flat, X, Y = _small_problem(seed=21)
    Wt = np.random.default_rng(2).uniform(0.1, 3.0, Y.shape)
    loss, g = mlp.loss_and_grad(flat, SMALL, X, Y, weights=Wt)
    h = 1e-6
    for k in range(0, flat.shape[0], 7):
        e = np.zeros_like(flat)
        e[k] = h
        fd = (mlp.loss_and_grad(flat + e, SMALL, X, Y, weights=Wt)[0]
              - mlp.loss_and_grad(flat - e, SMALL, X, Y, weights=Wt)[0]) / (2 * h)
        assert abs(g[k] - fd) < 1e-8 * max(1.0, abs(fd))
    yhat, _ = mlp.forward(flat, SMALL, X)
    assert loss == pytest.approx(np.mean(Wt * (yhat - Y) ** 2), rel=1e-15)
