"""FP64 reference of the emissivity surrogate (test infrastructure only).

The surrogate is not part of the paper's method: it is the learned
approximation the solver's users may swap in (the paper's introduction cites
precomputed emissivity tables as the cheap alternative it improves on).
This module fixes, in plain NumPy, what the GPU trainer and the fused
inference kernel compute, so that their gradients and outputs can be checked:

* features of a (field, grain) pair: log10 of the field's energy density in
  32 bands of the wavelength grid plus log10 of the grain radius (cm);
  band b spans grid nodes floor(b (L-1) / 32) .. floor((b+1) (L-1) / 32) and
  its energy is the trapezoid integral of u over those nodes;
* targets: y_lambda = log10(max(j_lambda, 1e-6 max j) / A), A the absorbed
  power of the pair on the grid (trapezoid of c u C_abs), then one more
  output y_L = log10(E / A), E = 4 pi int j dlambda (trapezoid) the emitted
  power: the plain model's own energy ratio (below 1 where coarse enthalpy
  bins leave photons near the grid's short end without a transition);
* the network: widths (33, 256, 256, 256, L + 1), GELU (erf form) after
  every hidden layer; inputs z-scored per column, targets centred per column,
  the L spectrum columns scaled by one pooled standard deviation and the
  ratio column by RATIO_SCALE times its own (a smaller weight in the loss);
* loss: mean squared error over samples and outputs; Adam updates;
* the accuracy metric: band-integrated j over the same 32 bands, relative
  error over the bands holding at least 1e-3 of the pair's emitted power.

``bf16=True`` rounds every matrix-product operand to bfloat16 (round to
nearest even) and keeps everything else in FP64: the GPU's BF16 products with
FP32 accumulation then differ from it only by accumulation order and by the
rare operand whose FP32 value rounds the other way.  In the forward pass the
input operand of the first and of the last layer is taken as two bfloat16
terms, hi = bf16(x) and lo = bf16(x - hi), each multiplied by the same
bfloat16 weights (a single bfloat16 keeps only 8 significant bits, which
blurs the band energies by about 1%); the backward products use one term.
"""

from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np
from scipy import special

N_BANDS = 32
SQRT2 = math.sqrt(2.0)
# forward layers whose input operand is split into two bfloat16 terms
SPLIT_LAYERS = (0, 3)
# scale of the energy-ratio target, in units of its own standard deviation
RATIO_SCALE = 10.0


# ---- features, targets, metric -------------------------------------------------

def band_edges(L: int) -> np.ndarray:
    return (np.arange(N_BANDS + 1) * (L - 1)) // N_BANDS


def band_integrals(f: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Trapezoid integral of f (..., L) over each band: (..., 32)."""
    e = band_edges(lam.shape[0])
    seg = 0.5 * (f[..., 1:] + f[..., :-1]) * np.diff(lam)
    csum = np.concatenate([np.zeros(f.shape[:-1] + (1,)), np.cumsum(seg, axis=-1)], axis=-1)
    return csum[..., e[1:]] - csum[..., e[:-1]]


def features(u: np.ndarray, lam: np.ndarray, radius_cm: float) -> np.ndarray:
    """Raw (un-normalised) inputs of one or more fields for one grain: (..., 33)."""
    E = band_integrals(np.asarray(u, dtype=np.float64), lam)
    x = np.log10(np.maximum(E, 1e-300))
    a = np.full(x.shape[:-1] + (1,), math.log10(radius_cm))
    return np.concatenate([x, a], axis=-1)


def emitted_power(j: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """4 pi int j dlambda over the grid (trapezoid): (...,)."""
    return 4.0 * math.pi * np.trapezoid(np.asarray(j, dtype=np.float64), lam, axis=-1)


def targets(j: np.ndarray, absorbed, lam: np.ndarray) -> np.ndarray:
    """Raw targets (..., L + 1): the floored log spectrum per absorbed power,
    then log10 of emitted over absorbed power."""
    j = np.asarray(j, dtype=np.float64)
    a = np.asarray(absorbed, dtype=np.float64)
    floor = 1e-6 * j.max(axis=-1, keepdims=True)
    spec = np.log10(np.maximum(j, floor) / a[..., None])
    ratio = np.log10(emitted_power(j, lam) / a)
    return np.concatenate([spec, ratio[..., None]], axis=-1)


def target_stats(Y: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Target normalisation of a training set Y [n, L + 1]: column means;
    one pooled standard deviation (root mean column variance) for the L
    spectrum columns, RATIO_SCALE times the ratio column's own for the last."""
    mu, sd = zscore_stats(Y)
    L = Y.shape[1] - 1
    s = sd.copy()
    s[:L] = math.sqrt(float(np.mean(sd[:L] ** 2)))
    s[L] *= RATIO_SCALE
    return mu, s


def band_rel_error(j: np.ndarray, jref: np.ndarray, lam: np.ndarray, min_share: float = 1e-3) -> np.ndarray:
    """Per pair: max over bands holding >= min_share of the reference's
    emitted power of |J_b / J_b,ref - 1|."""
    J = band_integrals(np.asarray(j, dtype=np.float64), lam)
    Jr = band_integrals(np.asarray(jref, dtype=np.float64), lam)
    tot = Jr.sum(axis=-1, keepdims=True)
    m = Jr >= min_share * tot
    err = np.where(m, np.abs(J / np.where(m, Jr, 1.0) - 1.0), 0.0)
    return err.max(axis=-1)


def band_node_weights(lam: np.ndarray) -> np.ndarray:
    """q [32, L]: the trapezoid weight of grid node k in band b, so that
    band_integrals(f) = q @ f."""
    L = lam.shape[0]
    e = band_edges(L)
    q = np.zeros((N_BANDS, L))
    for b in range(N_BANDS):
        for k in range(e[b], e[b + 1]):          # segment k .. k+1 lies in band b
            h = 0.5 * (lam[k + 1] - lam[k])
            q[b, k] += h
            q[b, k + 1] += h
    return q


def loss_weights(Y: np.ndarray, lam: np.ndarray, band_weight: float) -> np.ndarray:
    """Per-element weights W [n, L + 1] of the band-weighted loss from raw
    targets Y (log10 of j / A, then the ratio): with j_k = 10^y_k and J_b the
    band integrals, the bands counted are those with J_b >= 1e-3 sum J;
    rho_k = sum over counted b of j_k q_kb / J_b, divided by their number;
    W_k = (1 - band_weight) + band_weight L rho_k, and 1 for the ratio output.
    (An error d_k in log10 j_k changes J_b by ln 10 sum_k d_k j_k q_kb, so
    these weights put the loss where the band-integrated metric looks.)"""
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    L = lam.shape[0]
    q = band_node_weights(lam)
    j = 10.0 ** (Y[:, :L] - Y[:, :L].max(axis=1, keepdims=True))
    J = j @ q.T                                                   # [n, 32]
    on = J >= 1e-3 * J.sum(axis=1, keepdims=True)
    share = np.where(on, 1.0 / np.where(on, J, 1.0), 0.0)        # 1 / J_b on counted bands
    rho = j * (share @ q) / on.sum(axis=1, keepdims=True)
    W = np.ones_like(Y)
    W[:, :L] = (1.0 - band_weight) + band_weight * L * rho
    return W


# ---- network ----------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via the FP32 value."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isfinite(f), r, b)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _phi_cdf(z: np.ndarray) -> np.ndarray:
    # Phi(z) = (1 + erf(z / sqrt 2)) / 2, written with erfc so that the left
    # tail keeps its relative precision
    return 0.5 * special.erfc(-z / SQRT2)


def gelu(z: np.ndarray) -> np.ndarray:
    """z Phi(z), Phi the standard normal CDF (the exact, erf form of GELU)."""
    return z * _phi_cdf(z)


def gelu_grad(z: np.ndarray) -> np.ndarray:
    return _phi_cdf(z) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(flat: np.ndarray, widths: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat parameter vector -> [(W [out, in], b [out])] per layer."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = flat[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = flat[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == flat.shape[0]
    return out


def pack(layers: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def _mm(a: np.ndarray, b: np.ndarray, bf16: bool, split: bool = False) -> np.ndarray:
    if not bf16:
        return a @ b
    b = bf16_round(b)
    hi = bf16_round(a)
    if not split:
        return hi @ b
    # the low term is rounded from the FP32 residual, as on the device
    lo = bf16_round(np.asarray(a, dtype=np.float32) - hi.astype(np.float32))
    return hi @ b + lo @ b


def forward(flat: np.ndarray, widths: Sequence[int], X: np.ndarray, bf16: bool = False):
    """Network output for normalised inputs X [n, 33]; also the
    pre-activations and activations for the backward pass."""
    layers = unpack(flat, widths)
    h = np.asarray(X, dtype=np.float64)
    hs, zs = [h], []
    for i, (W, b) in enumerate(layers):
        z = _mm(h, W.T, bf16, split=i in SPLIT_LAYERS) + b
        zs.append(z)
        h = gelu(z) if i + 1 < len(layers) else z
        hs.append(h)
    return h, (hs, zs)


def loss_and_grad(flat: np.ndarray, widths: Sequence[int], X: np.ndarray, Y: np.ndarray, bf16: bool = False,
                  weights: np.ndarray = None):
    """L = mean over samples and outputs of W (yhat - y)^2 (W = 1 unless
    per-element weights are given) and dL/dparams (flat, same layout)."""
    layers = unpack(flat, widths)
    yhat, (hs, zs) = forward(flat, widths, X, bf16)
    n, m = yhat.shape
    r = yhat - Y
    W = np.ones_like(r) if weights is None else np.asarray(weights, dtype=np.float64)
    loss = float(np.mean(W * r * r))
    dz = 2.0 * W * r / (n * m)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        dW = _mm(dz.T, hs[i], bf16)
        db = dz.sum(axis=0)
        grads[i] = (dW, db)
        if i > 0:
            dh = _mm(dz, W, bf16)
            dz = dh * gelu_grad(zs[i - 1])
    return loss, pack(grads)


def grad_abs_terms(flat: np.ndarray, widths: Sequence[int], X: np.ndarray, Y: np.ndarray,
                   weights: np.ndarray = None) -> np.ndarray:
    """For every parameter, the sum of the absolute values of the terms whose
    sum is its gradient in the BF16-operand backward pass of loss_and_grad
    (same layout as the gradient): sum_n |bf16(dz_n,o)| |bf16(h_n,i)| for a
    weight, sum_n |dz_n,o| for a bias.  The scale of the rounding error of a
    gradient computed with other accumulation orders or an occasional operand
    rounded to the other BF16 neighbour (such a flip moves one term by at most
    one BF16 spacing, 2^-7 of the term)."""
    layers = unpack(flat, widths)
    yhat, (hs, zs) = forward(flat, widths, X, bf16=True)
    n, m = yhat.shape
    W = np.ones_like(yhat) if weights is None else np.asarray(weights, dtype=np.float64)
    dz = 2.0 * W * (yhat - Y) / (n * m)
    out = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        out[i] = (np.abs(bf16_round(dz)).T @ np.abs(bf16_round(hs[i])), np.abs(dz).sum(axis=0))
        if i > 0:
            dz = _mm(dz, W, True) * gelu_grad(zs[i - 1])
    return pack(out)


def output_abs_terms(flat: np.ndarray, widths: Sequence[int], X: np.ndarray) -> np.ndarray:
    """Per sample and output, the sum of the absolute values of the terms of
    the last layer's BF16 product (hi and lo terms of its split input) plus
    |bias|: the scale of the rounding error of an output computed with other
    accumulation orders or an occasional operand rounded the other way."""
    layers = unpack(flat, widths)
    _, (hs, _) = forward(flat, widths, X, bf16=True)
    W, b = layers[-1]
    h = hs[-2]
    hi = bf16_round(h)
    lo = bf16_round(np.asarray(h, dtype=np.float32) - hi.astype(np.float32))
    return (np.abs(hi) + np.abs(lo)) @ np.abs(bf16_round(W)).T + np.abs(b)


def adam_step(flat, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba), step number t >= 1.  Returns new
    (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def zscore_stats(A: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Column means and standard deviations (population); a constant column
    gets std 1."""
    A = np.asarray(A, dtype=np.float64)
    mu = A.mean(axis=0)
    sd = A.std(axis=0)
    return mu, np.where(sd > 0.0, sd, 1.0)
