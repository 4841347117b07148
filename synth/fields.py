"""Seeded radiation fields: sums of diluted blackbodies, optionally attenuated.

u_lambda(cell) = U * (4 pi / c) * sum_k W_k * jitter_k * B_lambda(T_k)
                 * exp(-tau_V * (lambda / 0.55 um)^-1.3)      [erg cm^-3 cm^-1]

T_k = 3000, 4000, 7500, 20000 K and W_k = 1e-13, 1.65e-13, 1e-14, 1e-16.
At U = 1 and no jitter the field's energy density integrates to 0.4627 eV
cm^-3, the ISRF normalisation the paper uses for its example fields (Sec.
2.3.1).

Random draws use numpy's PCG64 seeded per workload, in this order: U[n] (log-
uniform), then jitter[n, 4] (uniform in [1 - s, 1 + s]) if the recipe jitters,
then tau_V[n] (log-uniform) if the recipe attenuates.  Parameters are always
drawn for the full workload size and then indexed, so a reduced run sees the
same first cells as the full one.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

from .configs import CONSTANTS, MICRON_CM

BB_TEMPERATURES_K = np.array([3000.0, 4000.0, 7500.0, 20000.0])
BB_DILUTIONS = np.array([1.0e-13, 1.65e-13, 1.0e-14, 1.0e-16])


@dataclass(frozen=True)
class FieldRecipe:
    seed: int
    U_range: Tuple[float, float]
    jitter: float                                  # half-width of the uniform jitter (0 = none)
    tau_V_range: Optional[Tuple[float, float]]     # None = no attenuation


def _blackbody_lambda(lam_cm: np.ndarray, T: float) -> np.ndarray:
    h, c, k = CONSTANTS["h"], CONSTANTS["c"], CONSTANTS["k"]
    x = h * c / (lam_cm * k * T)
    with np.errstate(over="ignore"):
        return 2.0 * h * c * c / lam_cm ** 5 / np.expm1(x)


def field_parameters(recipe: FieldRecipe, n_total: int):
    """Per-cell draws (U, jitter[4], tau_V) for the whole workload."""
    rng = np.random.Generator(np.random.PCG64(recipe.seed))
    lo, hi = recipe.U_range
    U = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=n_total)
    if recipe.jitter > 0.0:
        jit = rng.uniform(1.0 - recipe.jitter, 1.0 + recipe.jitter, size=(n_total, 4))
    else:
        jit = np.ones((n_total, 4))
    if recipe.tau_V_range is not None:
        tlo, thi = recipe.tau_V_range
        tau = 10.0 ** rng.uniform(math.log10(tlo), math.log10(thi), size=n_total)
    else:
        tau = np.zeros(n_total)
    return U, jit, tau


def make_fields(lam_cm: np.ndarray, recipe: FieldRecipe, n_total: int,
                cells: Optional[np.ndarray] = None, chunk: int = 8192) -> np.ndarray:
    """Energy density u_lambda [len(cells), n_lambda] in erg cm^-3 cm^-1 (FP64)."""
    U, jit, tau = field_parameters(recipe, n_total)
    if cells is None:
        cells = np.arange(n_total)
    cells = np.asarray(cells, dtype=np.int64)
    c = CONSTANTS["c"]
    basis = np.stack([BB_DILUTIONS[k] * _blackbody_lambda(lam_cm, BB_TEMPERATURES_K[k])
                      for k in range(4)])                       # [4, L]
    ext_shape = (lam_cm / (0.55 * MICRON_CM)) ** (-1.3)         # [L]
    out = np.empty((cells.shape[0], lam_cm.shape[0]))
    for s in range(0, cells.shape[0], chunk):
        idx = cells[s:s + chunk]
        u = (jit[idx] @ basis) * (4.0 * math.pi / c) * U[idx, None]
        if recipe.tau_V_range is not None:
            u = u * np.exp(-tau[idx, None] * ext_shape[None, :])
        out[s:s + chunk] = u
    return out
