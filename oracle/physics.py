"""Physical building blocks of the oracle (FP64, CGS).  Test infrastructure only.

* Planck function B_lambda(T)                      (Sec. 2.3, eq:emission-lambda)
* Debye internal energy E(T) and its inverse T(E)  (Sec. 2.1: the bins are
  enthalpy bins; each carries the temperature its enthalpy corresponds to)
* absorption cross-section off the wavelength grid (Sec. 2.2, eq:cooling
  integrates sigma(E) over all photon energies up to E_f)
"""

from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, optimize

# CODATA 2018 exact values, CGS.  The oracle's own copy.
H = 6.62607015e-27          # erg s
C = 2.99792458e10           # cm s^-1
K = 1.380649e-16            # erg K^-1
EV = 1.602176634e-12        # erg
AMU = 1.66053906660e-24     # g
HC = H * C


def planck_lambda(lam_cm, T):
    """B_lambda(T) = 2 h c^2 / lambda^5 / (exp(hc / lambda k T) - 1),
    erg s^-1 cm^-2 sr^-1 cm^-1.  Written with expm1 so that the
    Rayleigh-Jeans side keeps full precision; overflow of the exponential on
    the Wien side gives exactly 0."""
    lam = np.asarray(lam_cm, dtype=np.float64)
    x = HC / (lam * K * np.asarray(T, dtype=np.float64))
    with np.errstate(over="ignore"):
        return 2.0 * H * C * C / lam ** 5 / np.expm1(x)


def _debye_integrand(x: float) -> float:
    if x < 1.0e-8:
        return x * x                       # x^3 / (e^x - 1) -> x^2 as x -> 0
    if x > 700.0:
        return 0.0
    return x ** 3 / math.expm1(x)


def debye_integral(y: float) -> float:
    """D(y) = int_0^y x^3 / (e^x - 1) dx by adaptive quadrature."""
    if y <= 0.0:
        return 0.0
    top = min(y, 200.0)                    # the integrand is below 1e-80 beyond 200
    with warnings.catch_warnings():
        # quad reports round-off when it cannot prove 2e-14; the closed-form
        # limits in the tests bound the actual error
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(_debye_integrand, 0.0, top, epsabs=0.0, epsrel=2.0e-14, limit=400)
    return val


def debye_energy(T: float, N: float, theta: float) -> float:
    """Vibrational energy of N atoms (3N Debye modes) at temperature T:
    E(T) = 9 N k T (T / theta)^3 D(theta / T)  [erg]  (reading R9)."""
    if T <= 0.0:
        return 0.0
    return 9.0 * N * K * T * (T / theta) ** 3 * debye_integral(theta / T)


def temperature_of_energy(E: float, N: float, theta: float) -> float:
    """Invert debye_energy by Brent's method on log T; relative tolerance at
    the double-precision floor."""
    if E <= 0.0:
        return 0.0
    # E(T) lies between the low-T form (3 pi^4 / 5) N k T^4 / theta^3 and 3 N k T,
    # which gives a bracket.
    T_hi_class = E / (3.0 * N * K)
    T_low_form = (E * theta ** 3 / ((3.0 * math.pi ** 4 / 5.0) * N * K)) ** 0.25
    lo = 0.5 * min(T_hi_class, T_low_form)
    hi = 2.0 * max(T_hi_class, T_low_form) + theta
    f = lambda lt: debye_energy(math.exp(lt), N, theta) - E
    lt = optimize.brentq(f, math.log(lo), math.log(hi), xtol=1.0e-300, rtol=1.0e-15, maxiter=500)
    return math.exp(lt)


def cross_section(lam_cm, lam_grid, cabs_table, longwave_index):
    """C_abs at arbitrary wavelengths from the grain's table (reading R10):
    log-log interpolation between grid nodes (the same rule the paper applies
    to the field in eq:interpolation), a power law lambda^-p beyond the long
    end, and the end value beyond the short end."""
    lam = np.atleast_1d(np.asarray(lam_cm, dtype=np.float64))
    lg = np.log(lam_grid)
    lc = np.log(cabs_table)
    out = np.empty_like(lam)
    inside = (lam >= lam_grid[0]) & (lam <= lam_grid[-1])
    out[inside] = np.exp(np.interp(np.log(lam[inside]), lg, lc))
    long_ = lam > lam_grid[-1]
    out[long_] = cabs_table[-1] * (lam[long_] / lam_grid[-1]) ** (-longwave_index)
    short = lam < lam_grid[0]
    out[short] = cabs_table[0]
    return out
