"""The table method in FP64 (test infrastructure only): the oracle's twin of
the library's precomputed-emissivity table.

The paper's introduction names precomputed emissivity tables, indexed by the
strength of the radiation field, as the cheap alternative to the full
stochastic solve.  Here such a table holds, for one grain, the full solve of
one reference field shape u_ref scaled to n_nodes strengths U_k (log-uniform
in log10 U between lo and hi), stored as y_k(lambda) = log2(j_lambda / A_k),
A_k the pair's absorbed power (so that a looked-up spectrum can carry the
absorbed power of the field it is applied to).  A field u is looked up by its
energy relative to the reference, U = int u dlambda / int u_ref dlambda (both
trapezoid on the grid, clamped to the node range), and gets
A(u) 2^((1 - w) y_k + w y_(k+1)) with k, w its position on the node grid; a
node value without emission (y = -inf) gives none unless the weight puts the
whole value on the other node.  The table's energy budget (the reference of
the surrogate's table check) is each node spectrum's emitted power per unit
absorbed power, interpolated linearly at a field's node coordinate.
"""

from __future__ import annotations

import math

import numpy as np

from .physics import C
from .model import solve_pair


def node_log10U(lo: float, hi: float, n_nodes: int) -> np.ndarray:
    return lo + np.arange(n_nodes) * (hi - lo) / (n_nodes - 1)


def absorbed_power(u: np.ndarray, cabs: np.ndarray, lam: np.ndarray) -> float:
    return float(np.trapezoid(C * np.asarray(u, dtype=np.float64) * cabs, lam))


def build_table(grain, lam: np.ndarray, u_ref: np.ndarray, lo: float, hi: float, n_nodes: int) -> np.ndarray:
    """y [n_nodes, L]: log2(j / A) of the solve of 10^x_k u_ref (-inf where j = 0)."""
    y = np.full((n_nodes, lam.shape[0]), -np.inf)
    for k, x in enumerate(node_log10U(lo, hi, n_nodes)):
        u = 10.0 ** x * np.asarray(u_ref, dtype=np.float64)
        _, j = solve_pair(u, grain, lam)
        A = absorbed_power(u, grain.cabs_cm2, lam)
        pos = j > 0.0
        y[k, pos] = np.log2(j[pos] / A)
    return y


def node_coordinate(u: np.ndarray, u_ref: np.ndarray, lam: np.ndarray, lo: float, hi: float, K: int):
    """Where field u sits on the node grid: t = (log10 U - lo) / step clamped
    to [0, K - 1], U = int u dlambda / int u_ref dlambda; returns the lower
    node k (at most K - 2) and the weight w = t - k of the upper one."""
    E = float(np.trapezoid(u, lam))
    Eref = float(np.trapezoid(u_ref, lam))
    t = (math.log10(E / Eref) - lo) / ((hi - lo) / (K - 1)) if E > 0.0 and Eref > 0.0 else 0.0
    t = min(max(t, 0.0), K - 1.0)
    k = min(int(math.floor(t)), K - 2)
    return k, t - k


def node_ratios(y: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """The energy budget of a table: for each node, the emitted power of its
    spectrum per unit absorbed power, 4 pi int 2^(y_k) dlambda (trapezoid on
    the grid; no emission where y_k = -inf)."""
    return 4.0 * math.pi * np.trapezoid(np.where(np.isfinite(y), np.exp2(y), 0.0), lam, axis=-1)


def budget_ratio(rho: np.ndarray, lo: float, hi: float, u: np.ndarray, u_ref: np.ndarray, lam: np.ndarray) -> float:
    """The budget's emitted / absorbed power for field u: the node ratios rho
    interpolated linearly at u's node coordinate."""
    k, w = node_coordinate(u, u_ref, lam, lo, hi, rho.shape[0])
    return float((1.0 - w) * rho[k] + w * rho[k + 1])


def lookup(y: np.ndarray, lo: float, hi: float, u: np.ndarray, u_ref: np.ndarray, cabs: np.ndarray,
           lam: np.ndarray) -> np.ndarray:
    """The table's spectrum for field u."""
    K = y.shape[0]
    k, w = node_coordinate(u, u_ref, lam, lo, hi, K)
    if w == 0.0:
        yy = y[k]
    elif w == 1.0:
        yy = y[k + 1]
    else:
        yy = (1.0 - w) * y[k] + w * y[k + 1]
    A = absorbed_power(u, cabs, lam)
    return A * np.exp2(yy)
