"""Workload definitions: wavelength grid, grain descriptions and field recipes.

Everything here is an *input* to the solve.  Units are CGS: lengths in cm,
energies in erg, cross-sections in cm^2.

The five workloads:

``c1_tiny``       1 carbonaceous grain, a = 10 A, 256 enthalpy bins log-spaced
                  1e-4 .. 10 eV, 400 wavelengths 0.09 .. 1000 um, 64 cells,
                  U log-uniform in [0.1, 1e3], no jitter.
``c2_batched``    32 carbonaceous radii log-spaced 3.5 .. 250 A (1024 bins at
                  3.5 A falling to 128 at 250 A), 500 wavelengths, 16384 cells,
                  U log-uniform in [0.1, 1e5], +-30 % jitter on each dilution.
``c3_uneven``     2 compositions (carbonaceous, silicate) x 64 radii
                  3.5 .. 2500 A, 65536 cells of c1-style fields attenuated by
                  exp(-tau_V (lambda / 0.55 um)^-1.3), tau_V log-uniform in
                  [0.01, 20].
``c4_train``      surrogate training set: 15625 c2-generator cells x the 64
                  c3 radii per composition (1e6 pairs) plus 1563 fresh cells
                  (100,032 pairs) held out, from a separate seed stream.
``c5_surrogate``  262144 c2-generator cells x 64 radii x 2 compositions.

Conventions that the paper leaves open and this package fixes (they are
inputs, shared verbatim by the oracle and the GPU path):

* absorption efficiency Q(lambda) = 1 / (1 + (lambda / 0.3 um)^p), p = 2 for
  carbonaceous and 1.5 for silicate grains, C_abs = pi a^2 Q;
* silicate mean atomic mass: MgFeSiO4 has 7 atoms and 172.23 amu, so 24.605
  amu per atom;
* enthalpy-grid end points for c2..c5 (the workloads give none): the lower end
  is the low-temperature Debye energy (3 pi^4 / 5) N k T^4 / theta^3 at
  T_lo = 5 K, or 2.5 K for c3, whose attenuated fields cool large silicate
  grains to an equilibrium temperature of 4.7 K (the grid must reach below the
  coldest equilibrium, else probability piles up in the lowest bin);
  the upper end is max(3 N k T_top, E_lo + 3 hc / lambda_min) with
  T_top = 511 K (carbonaceous) or 378 K (silicate), twice the equilibrium
  temperature of a large grain at U = 1e5, so that the top bin holds no
  probability even for the strongest field and the smallest grain can absorb
  three of the hardest photons;
* bin-count law for c2/c3: n = clamp(16 round(1024 (a / 3.5 A)^-q / 16), 128,
  1024) with q = ln 8 / ln(250 / 3.5), which gives 1024 bins at 3.5 A and 128
  at 250 A as the workload states, in multiples of 16.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

# CODATA 2018 exact values (CGS).  A private copy: the oracle and the HIP path
# each hold their own.
CONSTANTS = {
    "h": 6.62607015e-27,        # erg s
    "c": 2.99792458e10,         # cm s^-1
    "k": 1.380649e-16,          # erg K^-1
    "eV": 1.602176634e-12,      # erg
    "amu": 1.66053906660e-24,   # g
}

ANGSTROM_CM = 1.0e-8
MICRON_CM = 1.0e-4

LAMBDA_MIN_CM = 0.09 * MICRON_CM
LAMBDA_MAX_CM = 1000.0 * MICRON_CM

COMPOSITIONS = {
    # density g cm^-3, mean atom mass amu, Debye temperature K, Q exponent p,
    # top temperature of the enthalpy grid (K)
    "carbonaceous": dict(rho=2.2, m_atom_amu=12.0, theta_K=420.0, q_exponent=2.0, T_top=511.0),
    "silicate": dict(rho=3.5, m_atom_amu=172.232 / 7.0, theta_K=500.0, q_exponent=1.5, T_top=378.0),
}


def wavelength_grid_cm(n_lambda: int) -> np.ndarray:
    """Log-uniform wavelength grid from 0.09 um to 1000 um, both ends included."""
    j = np.arange(n_lambda, dtype=np.float64)
    return LAMBDA_MIN_CM * (LAMBDA_MAX_CM / LAMBDA_MIN_CM) ** (j / (n_lambda - 1))


def bins_for_radius(a_cm: float) -> int:
    """Bin-count law for the batched workloads (see module docstring)."""
    q = math.log(8.0) / math.log(250.0 / 3.5)
    n = 1024.0 * (a_cm / (3.5 * ANGSTROM_CM)) ** (-q)
    n = 16 * int(round(n / 16.0))
    return int(min(1024, max(128, n)))


@dataclass
class Grain:
    """One grain size of one composition, as handed to both solvers."""

    composition: str
    radius_cm: float
    rho: float
    m_atom_amu: float
    theta_K: float
    q_exponent: float
    n_bins: int
    E_lo_erg: float
    E_hi_erg: float
    cabs_cm2: np.ndarray            # [n_lambda] on the workload's wavelength grid
    longwave_index: float           # C_abs ~ lambda^-p beyond the grid's long end

    @property
    def n_atoms(self) -> float:
        m = self.m_atom_amu * CONSTANTS["amu"]
        return (4.0 * math.pi / 3.0) * self.radius_cm ** 3 * self.rho / m


def _cabs_table(a_cm: float, p: float, lam_cm: np.ndarray) -> np.ndarray:
    q = 1.0 / (1.0 + (lam_cm / (0.3 * MICRON_CM)) ** p)
    return math.pi * a_cm * a_cm * q


def _n_atoms(a_cm: float, rho: float, m_atom_amu: float) -> float:
    return (4.0 * math.pi / 3.0) * a_cm ** 3 * rho / (m_atom_amu * CONSTANTS["amu"])


def make_grain(composition: str, a_cm: float, lam_cm: np.ndarray, n_bins: int | None = None,
               E_range_erg: Tuple[float, float] | None = None, T_lo: float = 5.0) -> Grain:
    """Build a grain description; default bin count and enthalpy range follow
    the batched-workload conventions in the module docstring."""
    comp = COMPOSITIONS[composition]
    N = _n_atoms(a_cm, comp["rho"], comp["m_atom_amu"])
    k = CONSTANTS["k"]
    if E_range_erg is None:
        E_lo = (3.0 * math.pi ** 4 / 5.0) * N * k * T_lo ** 4 / comp["theta_K"] ** 3
        hc = CONSTANTS["h"] * CONSTANTS["c"]
        E_hi = max(3.0 * N * k * comp["T_top"], E_lo + 3.0 * hc / LAMBDA_MIN_CM)
    else:
        E_lo, E_hi = E_range_erg
    if n_bins is None:
        n_bins = bins_for_radius(a_cm)
    return Grain(
        composition=composition,
        radius_cm=float(a_cm),
        rho=comp["rho"],
        m_atom_amu=comp["m_atom_amu"],
        theta_K=comp["theta_K"],
        q_exponent=comp["q_exponent"],
        n_bins=int(n_bins),
        E_lo_erg=float(E_lo),
        E_hi_erg=float(E_hi),
        cabs_cm2=_cabs_table(a_cm, comp["q_exponent"], lam_cm),
        longwave_index=comp["q_exponent"],
    )


def radii_cm(a_min_A: float, a_max_A: float, n: int) -> np.ndarray:
    return ANGSTROM_CM * a_min_A * (a_max_A / a_min_A) ** (np.arange(n) / (n - 1.0))


@dataclass
class Workload:
    name: str
    config_id: int
    lam_cm: np.ndarray
    grains: List[Grain]
    n_cells: int
    field_recipe: "object"
    notes: Dict[str, object] = field(default_factory=dict)

    @property
    def n_lambda(self) -> int:
        return int(self.lam_cm.shape[0])

    @property
    def n_pairs(self) -> int:
        return self.n_cells * len(self.grains)


WORKLOAD_NAMES = ("c1_tiny", "c2_batched", "c3_uneven", "c4_train", "c5_surrogate")


def workload(name: str, n_cells: int | None = None) -> Workload:
    """Return a workload description.  ``n_cells`` overrides the cell count
    (for reduced test sizes); the seed stream is unchanged, so the first
    cells of a reduced workload equal the first cells of the full one."""
    from .fields import FieldRecipe

    eV = CONSTANTS["eV"]
    if name == "c1_tiny":
        lam = wavelength_grid_cm(400)
        g = make_grain("carbonaceous", 10.0 * ANGSTROM_CM, lam, n_bins=256,
                       E_range_erg=(1.0e-4 * eV, 10.0 * eV))
        rec = FieldRecipe(seed=4627000 + 1, U_range=(0.1, 1.0e3), jitter=0.0, tau_V_range=None)
        return Workload(name, 1, lam, [g], n_cells or 64, rec)
    if name == "c2_batched":
        lam = wavelength_grid_cm(500)
        gs = [make_grain("carbonaceous", a, lam) for a in radii_cm(3.5, 250.0, 32)]
        rec = FieldRecipe(seed=4627000 + 2, U_range=(0.1, 1.0e5), jitter=0.3, tau_V_range=None)
        return Workload(name, 2, lam, gs, n_cells or 16384, rec)
    if name == "c3_uneven":
        lam = wavelength_grid_cm(500)
        gs = [make_grain(c, a, lam, T_lo=2.5) for c in ("carbonaceous", "silicate")
              for a in radii_cm(3.5, 2500.0, 64)]
        rec = FieldRecipe(seed=4627000 + 3, U_range=(0.1, 1.0e3), jitter=0.0, tau_V_range=(0.01, 20.0))
        return Workload(name, 3, lam, gs, n_cells or 65536, rec)
    if name == "c4_train":
        lam = wavelength_grid_cm(500)
        gs = [make_grain(c, a, lam) for c in ("carbonaceous", "silicate")
              for a in radii_cm(3.5, 2500.0, 64)]
        rec = FieldRecipe(seed=4627000 + 4, U_range=(0.1, 1.0e5), jitter=0.3, tau_V_range=None)
        wl = Workload(name, 4, lam, gs, n_cells or 15625, rec)
        wl.notes["heldout_recipe"] = FieldRecipe(seed=4627000 + 40, U_range=(0.1, 1.0e5), jitter=0.3,
                                                 tau_V_range=None)
        wl.notes["heldout_cells"] = 1563
        return wl
    if name == "c5_surrogate":
        lam = wavelength_grid_cm(500)
        gs = [make_grain(c, a, lam) for c in ("carbonaceous", "silicate")
              for a in radii_cm(3.5, 2500.0, 64)]
        rec = FieldRecipe(seed=4627000 + 5, U_range=(0.1, 1.0e5), jitter=0.3, tau_V_range=None)
        return Workload(name, 5, lam, gs, n_cells or 262144, rec)
    raise KeyError(name)


def size_weights(radii_cm: np.ndarray, q: float = 3.5, per_H: float = 1.0e-25) -> np.ndarray:
    """Quadrature weights w_g of a power-law size distribution
    dn/da = K a^-q per H atom (the workloads' stand-in for a measured size
    distribution): the midpoint rule in ln a on the log-spaced radii,
    w_g = K a_g^(1-q) dln a (half weights at both ends), K = per_H x 1 cm^(q-1)."""
    a = np.asarray(radii_cm, dtype=np.float64)
    la = np.log(a)
    d = np.empty_like(a)
    if a.shape[0] == 1:
        d[:] = 1.0
    else:
        d[1:-1] = 0.5 * (la[2:] - la[:-2])
        d[0] = 0.5 * (la[1] - la[0])
        d[-1] = 0.5 * (la[-1] - la[-2])
    return per_H * a ** (1.0 - q) * d
