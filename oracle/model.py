"""The oracle's solve for one (radiation field, grain size) pair.  FP64, CGS.
Test infrastructure only.

Notation follows Porter & Vladimirov Sec. 2: M + 1 enthalpy bins i = 0..M,
transition matrix T_ij (rate from bin j to bin i), heating entries A_fi = T_fi
for f > i, cooling entries T_(f-1)f, cumulative matrix B, auxiliary vector X
and bin probabilities P.  The wavelength grid lambda_0..lambda_{L-1} is the
grid on which the field u_lambda and the cross-section C_abs are given.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Tuple

import numpy as np
from scipy import optimize

from .physics import H, C, K, HC, planck_lambda, temperature_of_energy, cross_section

RESCALE_THRESHOLD = 2.0 ** 500
RESCALE_FACTOR = 2.0 ** -500

_GL8 = np.polynomial.legendre.leggauss(8)
_GL16 = np.polynomial.legendre.leggauss(16)


@dataclass
class GrainSetup:
    """Field-independent per-grain quantities (Sec. 2.2: the cooling rates do
    not depend on the field and are precomputed)."""
    lam: np.ndarray          # [L] wavelength grid, cm
    cabs: np.ndarray         # [L] C_abs on the grid, cm^2
    longwave_index: float
    E: np.ndarray            # [M+1] bin enthalpies, erg
    dE: np.ndarray           # [M+1] bin widths, erg
    T: np.ndarray            # [M+1] bin temperatures, K
    cool: np.ndarray         # [M+1] T_(f-1)f for f >= 1 (cool[0] = 0), s^-1
    planck: np.ndarray       # [M+1, L] B_lambda(T_i) * [E_i >= hc / lambda], cgs per sr


def enthalpy_grid(E_lo: float, E_hi: float, n_bins: int) -> Tuple[np.ndarray, np.ndarray]:
    """Log-uniform enthalpy grid E_i = E_lo (E_hi / E_lo)^(i / M), i = 0..M, and
    bin widths dE_i = E_i (r^(1/2) - r^(-1/2)) with r = (E_hi / E_lo)^(1 / M):
    bin i spans the geometric midpoints to its neighbours (reading R8; Sec. 2.1
    only requires narrow bins)."""
    M = n_bins - 1
    i = np.arange(n_bins, dtype=np.float64)
    E = E_lo * (E_hi / E_lo) ** (i / M)
    r = (E_hi / E_lo) ** (1.0 / M)
    dE = E * (math.sqrt(r) - 1.0 / math.sqrt(r))
    return E, dE


def _panels(a: float, b: float, width: float, rule):
    n = max(1, int(math.ceil((b - a) / width)))
    edges = np.linspace(a, b, n + 1)
    mid = 0.5 * (edges[1:] + edges[:-1])
    half = 0.5 * (edges[1:] - edges[:-1])
    x = (mid[:, None] + half[:, None] * rule[0][None, :]).ravel()
    w = (half[:, None] * rule[1][None, :]).ravel()
    return x, w


def cooling_integral(E_f: float, T_f: float, lam: np.ndarray, cabs: np.ndarray, p_long: float) -> float:
    """int_0^{E_f} E^3 C_abs(hc/E) / (exp(E / k T_f) - 1) dE  (Sec. 2.2, eq:cooling).

    The integral runs over all photon energies up to E_f, not only those on
    the wavelength grid (reading R3): otherwise bins below hc / lambda_max would
    get no cooling.  It is taken in u = ln E with Gauss-Legendre rules on the
    pieces where the integrand is smooth: each wavelength-grid interval (where
    C_abs is a power law, reading R10), the long-wave power-law tail, and the
    short-wave constant-C_abs tail."""
    kT = K * T_f
    E_nodes = HC / lam[::-1]                          # ascending photon energies of the grid nodes
    pts, wts = [], []
    u_top = math.log(E_f)
    # photons softer than the grid: power-law C_abs
    u0 = math.log(E_nodes[0])
    hi = min(u0, u_top)
    x, w = _panels(hi - 40.0, hi, 1.0, _GL16)
    pts.append(x); wts.append(w)
    # grid intervals
    for m in range(E_nodes.shape[0] - 1):
        a, b = math.log(E_nodes[m]), math.log(E_nodes[m + 1])
        if a >= u_top:
            break
        b = min(b, u_top)
        x, w = _panels(a, b, 1.0, _GL8)
        pts.append(x); wts.append(w)
    # photons harder than the grid: constant C_abs
    if u_top > math.log(E_nodes[-1]):
        a = math.log(E_nodes[-1])
        b = min(u_top, math.log(800.0 * kT)) if 800.0 * kT > E_nodes[-1] else a
        if b > a:
            x, w = _panels(a, b, 0.05, _GL8)
            pts.append(x); wts.append(w)
    u = np.concatenate(pts)
    wt = np.concatenate(wts)
    E = np.exp(u)
    sig = cross_section(HC / E, lam, cabs, p_long)
    with np.errstate(over="ignore"):
        occ = 1.0 / np.expm1(E / kT)
    f = E ** 4 * sig * occ                              # E^3 sigma / (e^x - 1), times dE/du = E
    return float(np.sum(wt * f))


def cooling_rates(E: np.ndarray, T: np.ndarray, lam, cabs, p_long) -> np.ndarray:
    """T_(f-1)f = [1 / (E_f - E_(f-1))] (8 pi / (h^3 c^2)) int_0^{E_f} E^3 sigma /
    (e^{E/kT_f} - 1) dE for f >= 1  (Sec. 2.2, eq:cooling with the constant read
    as 8 pi / (h^3 c^2), reading R3: emitted power per energy step)."""
    out = np.zeros_like(E)
    pref = 8.0 * math.pi / (H ** 3 * C ** 2)
    for f in range(1, E.shape[0]):
        out[f] = pref * cooling_integral(E[f], T[f], lam, cabs, p_long) / (E[f] - E[f - 1])
    return out


def planck_table(T: np.ndarray, E: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """B_lambda(T_i) [E_i >= h nu], the bracket of eq:emission-lambda without
    the stray P_i (reading R4): a grain in bin i cannot emit a photon with more
    energy than it holds."""
    tab = planck_lambda(lam[None, :], T[:, None])
    allowed = E[:, None] >= HC / lam[None, :]
    return np.where(allowed, tab, 0.0)


_SETUP_CACHE: Dict[tuple, GrainSetup] = {}


def _setup_key(grain, lam: np.ndarray) -> tuple:
    return (grain.composition, grain.radius_cm, grain.n_bins, grain.E_lo_erg, grain.E_hi_erg,
            grain.theta_K, grain.n_atoms, lam.shape[0], float(lam[0]), float(lam[-1]),
            float(grain.cabs_cm2[0]), float(grain.cabs_cm2[-1]), grain.longwave_index)


def preload_setup(grain, lam: np.ndarray, setup: GrainSetup) -> None:
    """Put a setup computed elsewhere (another process) into the cache."""
    _SETUP_CACHE[_setup_key(grain, lam)] = setup


def grain_setup(grain, lam: np.ndarray) -> GrainSetup:
    """Per-grain precompute: enthalpy grid, bin temperatures from the Debye
    heat capacity, cooling rates and the Planck table.  Cached per grain."""
    key = _setup_key(grain, lam)
    hit = _SETUP_CACHE.get(key)
    if hit is not None:
        return hit
    E, dE = enthalpy_grid(grain.E_lo_erg, grain.E_hi_erg, grain.n_bins)
    N = grain.n_atoms
    T = np.array([temperature_of_energy(e, N, grain.theta_K) for e in E])
    cabs = np.asarray(grain.cabs_cm2, dtype=np.float64)
    cool = cooling_rates(E, T, lam, cabs, grain.longwave_index)
    planck = planck_table(T, E, lam)
    s = GrainSetup(lam=lam, cabs=cabs, longwave_index=grain.longwave_index, E=E, dE=dE, T=T,
                   cool=cool, planck=planck)
    _SETUP_CACHE[key] = s
    return s


def absorbed_cumulative(u: np.ndarray, setup: GrainSetup) -> np.ndarray:
    """Cum_j = int_{lambda_j}^{lambda_{L-1}} c u C_abs dlambda by the trapezoid rule
    over grid nodes (absorbed power from photons at wavelengths >= lambda_j)."""
    rho = C * u * setup.cabs
    seg = 0.5 * (rho[1:] + rho[:-1]) * np.diff(setup.lam)
    cum = np.zeros_like(rho)
    cum[:-1] = np.cumsum(seg[::-1])[::-1]
    return cum


def _first_at_least(lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Index of the first grid wavelength >= x (L if none)."""
    return np.searchsorted(lam, x, side="left")


def heating_matrix(u: np.ndarray, setup: GrainSetup, intrabin: bool = True) -> np.ndarray:
    """Dense heating block A[f, i] = T_fi for f > i (zero elsewhere).

    Sec. 2.2: T_ul = Omega(lambda) lambda^3 dE / (h^2 c) with Omega = u_lambda C_abs
    interpolated log-log between the bracketing grid wavelengths
    (eq:heating, eq:interpolation).  Readings: R1 (constant h^2 c: photon
    counting with u an energy density per unit wavelength), R2 (dE is the
    width of the upper bin f), R5 (bracket j = first grid index with
    lambda_j >= lambda, clamped to [1, L-1]; zero rate outside the grid or
    when an end point is not positive), R11 (no transitions above the top bin).

    ``intrabin`` adds, to the adjacent entry A[i+1, i], the absorbed power of
    photons too soft to reach bin i+1 divided by E_(i+1) - E_i (reading R6,
    the continuous-heating term of Draine & Li that the paper omits)."""
    lam = setup.lam
    L = lam.shape[0]
    E, dE = setup.E, setup.dE
    n = E.shape[0]
    omega = u * setup.cabs
    f_idx, i_idx = np.tril_indices(n, k=-1)             # f > i
    eps = E[f_idx] - E[i_idx]
    lam_fi = HC / eps
    inside = (lam_fi >= lam[0]) & (lam_fi <= lam[-1])
    j = np.clip(_first_at_least(lam, lam_fi), 1, L - 1)
    lo = omega[j - 1]
    hi = omega[j]
    ok = inside & (lo > 0.0) & (hi > 0.0)
    rate = np.zeros_like(eps)
    jj, lf, lo_, hi_ = j[ok], lam_fi[ok], lo[ok], hi[ok]
    w = np.log(lf / lam[jj - 1]) / np.log(lam[jj] / lam[jj - 1])
    om = np.exp(np.log(lo_) + w * (np.log(hi_) - np.log(lo_)))
    rate[ok] = om * lf ** 3 * dE[f_idx[ok]] / (H * H * C)
    A = np.zeros((n, n))
    A[f_idx, i_idx] = rate
    if intrabin:
        cum = absorbed_cumulative(u, setup)
        for i in range(n - 1):
            gap = E[i + 1] - E[i]
            if gap > HC / lam[0]:
                jstar = 0                                   # every grid photon is softer than the step
            else:
                eps_lo = (E[i + 1] - 0.5 * dE[i + 1]) - E[i]
                # eps_lo <= 0: the discrete step already covers every photon energy
                jstar = int(_first_at_least(lam, np.array([HC / eps_lo]))[0]) if eps_lo > 0 else L
            if jstar < L:
                A[i + 1, i] += cum[jstar] / gap
    return A


def b_matrix_recurrence(A: np.ndarray) -> np.ndarray:
    """B_fj = sum_{k=f}^{M} A_kj for f > j (eq:bmatrix), built from the top
    row down by B_fj = B_(f+1)j + A_fj (eq:brecurrence).  Entries with f <= j
    are zero."""
    n = A.shape[0]
    B = np.zeros_like(A)
    run = np.zeros(n)
    for f in range(n - 1, 0, -1):
        run[:f] += A[f, :f]
        B[f, :f] = run[:f]
    return B


def b_matrix_triple_sum(A: np.ndarray) -> np.ndarray:
    """B by the explicit sum of eq:bmatrix (O(M^3)); for checking the recurrence."""
    n = A.shape[0]
    B = np.zeros_like(A)
    for f in range(1, n):
        for j in range(f):
            s = 0.0
            for k in range(f, n):
                s += A[k, j]
            B[f, j] = s
    return B


def recursion(B: np.ndarray, cool: np.ndarray, threshold: float = RESCALE_THRESHOLD,
              factor: float = RESCALE_FACTOR):
    """X_0 = 1, X_f = (1 / T_(f-1)f) sum_{j<f} B_fj X_j (eq:xf), then
    P = X / sum X (eq:renormalization).

    Whenever a new X_f exceeds ``threshold`` the whole vector X_0..X_f is
    multiplied by ``factor`` (the appendix on precision control rescales by
    1e-30 above 1e30 in single precision; in double precision a power of two
    2^-500 above 2^500 keeps the rescale exact, reading R7).
    Returns (P, X, n_rescales)."""
    n = B.shape[0]
    X = np.zeros(n)
    X[0] = 1.0
    n_rescale = 0
    for f in range(1, n):
        X[f] = np.dot(B[f, :f], X[:f]) / cool[f]
        if X[f] > threshold:
            X[:f + 1] *= factor
            n_rescale += 1
    P = X / np.sum(X)
    return P, X, n_rescale


def emission(P: np.ndarray, setup: GrainSetup) -> np.ndarray:
    """j_lambda = C_abs(lambda) sum_i P_i B_lambda(T_i) [E_i >= hc / lambda]
    (Sec. 2.3, eq:emission and eq:emission-lambda read per unit wavelength and
    per steradian, reading R4).  erg s^-1 sr^-1 cm^-1 per grain."""
    return setup.cabs * (P @ setup.planck)


def diagnostics(u: np.ndarray, setup: GrainSetup, P: np.ndarray, j: np.ndarray, A: np.ndarray):
    """Energy bookkeeping for one pair (reading R12):

    absorbed   int c u C_abs dlambda over the grid (trapezoid)
    emitted    4 pi int j_lambda dlambda over the grid (trapezoid)
    A_rep      sum_i P_i int_{eps <= E_M + dE_M/2 - E_i} c u C_abs dlambda: the
               absorbed power the discrete model can represent (photons that
               would lift the grain above the top bin are dropped)
    heat, cool discrete heating and cooling power of the steady state,
               sum_i P_i sum_{f>i} A_fi (E_f - E_i) and sum_f P_f T_(f-1)f (E_f - E_(f-1));
               equal for the exact steady state."""
    lam = setup.lam
    E, dE = setup.E, setup.dE
    cum = absorbed_cumulative(u, setup)
    absorbed = float(cum[0])
    emitted = float(4.0 * math.pi * np.trapezoid(j, lam))
    top = E[-1] + 0.5 * dE[-1]
    edge = top - E
    jrep = np.where(edge > 0.0, _first_at_least(lam, HC / np.where(edge > 0.0, edge, 1.0)), lam.shape[0])
    cum_ext = np.append(cum, 0.0)
    A_rep = float(np.sum(P * cum_ext[np.minimum(jrep, lam.shape[0])]))
    dEm = E[:, None] - E[None, :]
    heat = float(np.sum(P[None, :] * A * np.where(dEm > 0, dEm, 0.0)))
    coolp = float(np.sum(P[1:] * setup.cool[1:] * (E[1:] - E[:-1])))
    return {"absorbed": absorbed, "emitted": emitted, "A_rep": A_rep, "heat": heat, "cool": coolp}


def solve_pair(u: np.ndarray, grain, lam: np.ndarray, intrabin: bool = True,
               threshold: float = RESCALE_THRESHOLD, with_diag: bool = False):
    """Full plain solve for one pair: rates -> B -> recursion -> P -> j_lambda."""
    setup = grain_setup(grain, lam)
    A = heating_matrix(u, setup, intrabin=intrabin)
    B = b_matrix_recurrence(A)
    P, X, nres = recursion(B, setup.cool, threshold=threshold)
    j = emission(P, setup)
    if with_diag:
        d = diagnostics(u, setup, P, j, A)
        d["n_rescale"] = nres
        return P, j, d
    return P, j


def equilibrium_temperature(u: np.ndarray, setup: GrainSetup) -> float:
    """T_eq with int c u C dlambda = 4 pi int C B_lambda(T) dlambda on the grid
    (trapezoid), the thermal-equilibrium temperature a large grain collapses to."""
    lam = setup.lam
    absorbed = float(np.trapezoid(C * u * setup.cabs, lam))
    g = lambda lt: 4.0 * math.pi * float(np.trapezoid(setup.cabs * planck_lambda(lam, math.exp(lt)), lam)) - absorbed
    return math.exp(optimize.brentq(g, math.log(1.0), math.log(1.0e5), xtol=1e-14, rtol=1e-14))


def size_convolution(j: np.ndarray, weights: np.ndarray, lam: np.ndarray, lambda_weighted: bool = True) -> np.ndarray:
    """Sec. 2.3, eq:convolution on a discrete size grid: the emissivity of the
    whole size distribution, sum_g w_g j_lambda(a_g), with w_g the quadrature
    weights of the distribution (per H atom); times lambda when
    lambda_weighted, giving lambda j_lambda = nu j_nu, the form the paper's
    library returns (its interface section).  j: [..., G, L]."""
    s = np.einsum("...gl,g->...l", np.asarray(j, dtype=np.float64), np.asarray(weights, dtype=np.float64))
    return s * lam if lambda_weighted else s
