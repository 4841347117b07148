"""Pins of the oracle's physical building blocks against closed forms and
limits fixed by the mathematics (CPU only)."""

import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import model as om
from oracle.physics import H, C, K, HC


def test_planck_integral_is_stefan_boltzmann():
    # int B_lambda dlambda = sigma T^4 / pi, sigma = 2 pi^5 k^4 / (15 c^2 h^3)
    sigma = 2.0 * math.pi ** 5 * K ** 4 / (15.0 * C ** 2 * H ** 3)
    for T in (30.0, 300.0, 6000.0):
        lam_peak = 0.2898 / T
        lam = np.geomspace(lam_peak * 1e-2, lam_peak * 1e4, 200001)
        val = np.trapezoid(oracle.planck_lambda(lam, T), lam)
        assert abs(val / (sigma * T ** 4 / math.pi) - 1.0) < 1e-7


def test_planck_limits():
    T = 100.0
    lam = 10.0                                   # hc / lambda k T ~ 1.4e-3: Rayleigh-Jeans
    rj = 2.0 * C * K * T / lam ** 4
    x = HC / (lam * K * T)
    assert abs(oracle.planck_lambda(lam, T) / rj - (x / math.expm1(x))) < 1e-14
    lam = 1e-6                                   # x ~ 1.4e4: exp overflows -> exactly 0 on the Wien side
    assert oracle.planck_lambda(np.array([lam]), 1.0)[0] == 0.0
    lam = 1e-4; T = 50.0                         # Wien
    x = HC / (lam * K * T)
    wien = 2.0 * H * C * C / lam ** 5 * math.exp(-x)
    assert abs(oracle.planck_lambda(lam, T) / wien - 1.0) < 1e-12


@pytest.mark.parametrize("theta", [420.0, 500.0])
def test_debye_low_temperature_limit(theta):
    N = 1234.5
    T = theta / 2000.0
    low = (3.0 * math.pi ** 4 / 5.0) * N * K * T ** 4 / theta ** 3
    assert abs(oracle.debye_energy(T, N, theta) / low - 1.0) < 1e-12


@pytest.mark.parametrize("theta", [420.0, 500.0])
def test_debye_high_temperature_expansion(theta):
    # E = 3 N k T [1 - 3x/8 + x^2/20 - x^4/1680 + ...], x = theta / T
    N = 77.0
    T = 50.0 * theta
    x = theta / T
    series = 3.0 * N * K * T * (1.0 - 3.0 * x / 8.0 + x * x / 20.0 - x ** 4 / 1680.0)
    assert abs(oracle.debye_energy(T, N, theta) / series - 1.0) < 1e-12


def test_debye_heat_capacity_against_quadrature_of_cv():
    # dE/dT equals the Debye heat capacity 9 N k (T/theta)^3 int_0^{theta/T} x^4 e^x / (e^x - 1)^2 dx
    N, theta, T = 500.0, 420.0, 60.0
    y = theta / T
    cv = 9.0 * N * K * (T / theta) ** 3 * integrate.quad(
        lambda x: x ** 4 * math.exp(x) / math.expm1(x) ** 2, 0.0, y, epsrel=1e-13)[0]
    h = 1e-4 * T
    dEdT = (oracle.debye_energy(T + h, N, theta) - oracle.debye_energy(T - h, N, theta)) / (2 * h)
    assert abs(dEdT / cv - 1.0) < 1e-8


def test_temperature_inversion_round_trip():
    N, theta = 462.5, 420.0
    for E in np.geomspace(1e-4, 1e3, 15) * oracle.EV:
        T = oracle.temperature_of_energy(E, N, theta)
        assert abs(oracle.debye_energy(T, N, theta) / E - 1.0) < 1e-13


def test_ten_angstrom_scale():
    # a = 10 A carbonaceous grain: N ~ 462.5; 1e-4 eV <-> ~7.5 K, 10 eV <-> ~199 K
    import synth
    w = synth.workload("c1_tiny")
    g = w.grains[0]
    assert abs(g.n_atoms - 462.5) < 0.5
    T0 = oracle.temperature_of_energy(1e-4 * oracle.EV, g.n_atoms, g.theta_K)
    T1 = oracle.temperature_of_energy(10.0 * oracle.EV, g.n_atoms, g.theta_K)
    assert 7.4 < T0 < 7.6 and 198.0 < T1 < 200.0


def test_cross_section_nodes_and_power_laws():
    lam = np.geomspace(1e-5, 0.1, 60)
    tab = 3.0e-14 * (lam / 1e-4) ** -1.7
    # exact at nodes
    assert np.allclose(oracle.cross_section(lam, lam, tab, 1.7), tab, rtol=1e-14, atol=0)
    # log-log interpolation of a power law is exact between nodes
    x = np.geomspace(1.1e-5, 0.09, 333)
    assert np.allclose(oracle.cross_section(x, lam, tab, 1.7), 3.0e-14 * (x / 1e-4) ** -1.7, rtol=1e-12, atol=0)
    # long-wave extrapolation continues the power law; short-wave is flat
    y = np.array([0.5, 3.0])
    assert np.allclose(oracle.cross_section(y, lam, tab, 1.7), 3.0e-14 * (y / 1e-4) ** -1.7, rtol=1e-12, atol=0)
    assert np.allclose(oracle.cross_section(np.array([1e-6]), lam, tab, 1.7), tab[0], rtol=0, atol=0)


def test_cooling_integral_power_law_closed_form():
    # sigma = C0 E^p everywhere -> int_0^inf E^(3+p) / (e^(E/kT) - 1) dE = (kT)^(4+p) Gamma(4+p) zeta(4+p)
    import synth
    p = 2.0
    lam = synth.wavelength_grid_cm(400)
    C0 = 1e-12
    tab = C0 * (HC / lam) ** p
    for T in (8.0, 120.0, 900.0):
        kT = K * T
        E_f = 300.0 * kT
        got = om.cooling_integral(E_f, T, lam, tab, p)
        # above the grid's short end the table is flat: integrate the correction exactly
        E_top = HC / lam[0]
        corr = integrate.quad(lambda E: E ** 3 * (C0 * E_top ** p - C0 * E ** p) / math.expm1(E / kT),
                              E_top, max(E_top, E_f), epsrel=1e-12)[0] if E_f > E_top else 0.0
        exact = C0 * kT ** (4 + p) * special.gamma(4 + p) * special.zeta(4 + p) + corr
        assert abs(got / exact - 1.0) < 1e-11


def test_cooling_integral_against_adaptive_quadrature():
    import synth
    w = synth.workload("c2_batched", n_cells=1)
    g = w.grains[5]
    lam = w.lam_cm
    for E_f, T in ((1e-3 * oracle.EV, 12.0), (2.0 * oracle.EV, 300.0), (30.0 * oracle.EV, 2500.0)):
        got = om.cooling_integral(E_f, T, lam, g.cabs_cm2, g.longwave_index)
        kT = K * T
        f = lambda lnE: (math.exp(lnE) ** 4 * oracle.cross_section(np.array([HC / math.exp(lnE)]), lam,
                         g.cabs_cm2, g.longwave_index)[0] / math.expm1(math.exp(lnE) / kT))
        pts = [math.log(HC / l) for l in lam if HC / l < E_f]
        lo = math.log(min(E_f, HC / lam[-1])) - 40.0
        ref = 0.0
        edges = [lo] + sorted(pts) + [math.log(E_f)]
        for a, b in zip(edges[:-1], edges[1:]):
            if b > a:
                ref += integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)[0]
        assert abs(got / ref - 1.0) < 1e-11
