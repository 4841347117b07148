"""Seeded initial weights of the emissivity surrogate (an input, like the
fields): the random numbers training starts from, drawn once here and handed
to the GPU trainer and to the FP64 reference MLP alike.

Layout of the flat FP32 vector, layer by layer for the widths
(33, 256, 256, 256, n_out): W_l as a row-major [out][in] matrix, then b_l.
W_l is uniform in [-s, s] with s = sqrt(6 / in) (He-uniform, suited to GELU);
biases start at 0.
"""

from __future__ import annotations

import numpy as np

HIDDEN = (256, 256, 256)
N_IN = 33


def n_outputs(n_lambda: int) -> int:
    """Network outputs for a spectrum of n_lambda wavelengths: the spectrum,
    then the energy ratio."""
    return int(n_lambda) + 1


def widths(n_out: int):
    return (N_IN,) + HIDDEN + (int(n_out),)


def n_params(n_out: int) -> int:
    w = widths(n_out)
    return sum(w[i + 1] * w[i] + w[i + 1] for i in range(len(w) - 1))


def init_params(n_out: int, seed: int = 4627004) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    w = widths(n_out)
    parts = []
    for i in range(len(w) - 1):
        s = np.sqrt(6.0 / w[i])
        parts.append(rng.uniform(-s, s, size=w[i + 1] * w[i]).astype(np.float32))
        parts.append(np.zeros(w[i + 1], dtype=np.float32))
    return np.concatenate(parts)
