"""Dense steady-state solve of the master equation.  Test infrastructure only.

Sec. 2.1: sum_{j != i} T_ij P_j - sum_{j != i} T_ji P_i = 0 for every bin i
(eq:steady-state) with sum_i P_i = 1 (eq:level-sum).  In the thermal
continuous approximation the only downward entries are T_(f-1)f (eq:adjacent).
This solves the full (M+1) x (M+1) system with one balance equation replaced by
the normalisation, by LU factorisation.  The paper notes that the diagonal of
this direct form is a difference of nearly equal positive numbers; to keep the
check independent of that cancellation the LU solve runs in multiple-precision
arithmetic (mpmath, 60 significant digits by default), so it is only used at
small bin counts.
"""

from __future__ import annotations

import mpmath
import numpy as np


def transition_matrix(A: np.ndarray, cool: np.ndarray) -> np.ndarray:
    """T[i, j] = rate j -> i: heating A[f, i] below the diagonal, cooling
    cool[f] = T_(f-1)f on the first superdiagonal."""
    n = A.shape[0]
    T = np.tril(A, k=-1).copy()
    for f in range(1, n):
        T[f - 1, f] = cool[f]
    return T


def dense_steady_state(A: np.ndarray, cool: np.ndarray, digits: int = 60) -> np.ndarray:
    T = transition_matrix(A, cool)
    n = T.shape[0]
    with mpmath.workdps(digits):
        Tm = mpmath.matrix([[mpmath.mpf(float(T[i, j])) for j in range(n)] for i in range(n)])
        Lm = mpmath.matrix(n, n)
        for j in range(n):
            out = mpmath.fsum(Tm[i, j] for i in range(n))          # total rate out of bin j
            for i in range(n):
                Lm[i, j] = Tm[i, j] - (out if i == j else 0)
        for j in range(n):
            Lm[n - 1, j] = 1                                        # sum P = 1 replaces the last row
        rhs = mpmath.matrix([0] * (n - 1) + [1])
        P = mpmath.lu_solve(Lm, rhs)
        return np.array([float(P[i]) for i in range(n)])
