"""Pins of the oracle's solve: B matrix, recursion, rates, emission and energy
balance, against brute force, closed forms, special cases and invariants
(CPU only)."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import model as om
from oracle.physics import H, C, K, HC
from synth.fields import make_fields, FieldRecipe


def _random_rates(n, rng, decades=6):
    A = np.tril(10.0 ** rng.uniform(-decades, 0, size=(n, n)), k=-1)
    cool = np.zeros(n)
    cool[1:] = 10.0 ** rng.uniform(-3, 1, size=n - 1)
    return A, cool


def test_b_recurrence_equals_triple_sum():
    rng = np.random.default_rng(1)
    A, _ = _random_rates(13, rng)
    Br = om.b_matrix_recurrence(A)
    Bt = om.b_matrix_triple_sum(A)
    assert np.allclose(Br, Bt, rtol=1e-14, atol=0)
    # nothing on or above the diagonal
    assert np.all(np.triu(Br) == 0.0)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_recursion_equals_dense_master_equation(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        A, cool = _random_rates(n, rng)
        P, _, _ = om.recursion(om.b_matrix_recurrence(A), cool)
        Pd = oracle.dense_steady_state(A, cool)
        assert np.allclose(P, Pd, rtol=1e-13, atol=0)
        assert abs(P.sum() - 1.0) < 1e-15


def test_two_bin_closed_form():
    A = np.array([[0.0, 0.0], [3.7e-3, 0.0]])
    cool = np.array([0.0, 2.9e-2])
    P, _, _ = om.recursion(om.b_matrix_recurrence(A), cool)
    p1 = 3.7e-3 / (3.7e-3 + 2.9e-2)
    assert abs(P[1] / p1 - 1.0) < 4e-16 and abs(P[0] / (1.0 - p1) - 1.0) < 4e-16


def test_dense_matrix_is_thermal_continuous():
    rng = np.random.default_rng(7)
    A, cool = _random_rates(9, rng)
    from oracle.dense import transition_matrix
    T = transition_matrix(A, cool)
    # eq:adjacent: T_ij = 0 for i < j - 1
    for i in range(9):
        for j in range(9):
            if i < j - 1:
                assert T[i, j] == 0.0


@pytest.fixture(scope="module")
def c1():
    w = synth.workload("c1_tiny")
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells)
    setup = oracle.grain_setup(w.grains[0], w.lam_cm)
    return w, u, setup


def test_recursion_matches_dense_on_physical_rates():
    # a tiny physical grain with 16 bins: the dense LU solve of the full master
    # equation agrees with the recursion
    lam = synth.wavelength_grid_cm(400)
    g = synth.make_grain("carbonaceous", 6.0e-8, lam, n_bins=16, E_range_erg=(0.05 * oracle.EV, 40.0 * oracle.EV))
    u = make_fields(lam, FieldRecipe(9, (1.0, 1.0), 0.0, None), 1)[0]
    s = oracle.grain_setup(g, lam)
    A = om.heating_matrix(u, s)
    P, _, _ = om.recursion(om.b_matrix_recurrence(A), s.cool)
    Pd = oracle.dense_steady_state(A, s.cool)
    assert np.allclose(P, Pd, rtol=1e-13, atol=0)


def test_sum_P_and_rescale_invariance(c1):
    w, u, s = c1
    for c in range(0, 64, 9):
        A = om.heating_matrix(u[c], s)
        B = om.b_matrix_recurrence(A)
        P1, _, n1 = om.recursion(B, s.cool)
        P2, _, n2 = om.recursion(B, s.cool, threshold=2.0 ** 20, factor=2.0 ** -20)
        assert n2 > n1
        assert abs(P1.sum() - 1.0) < 1e-14
        big = P1 > 1e-250
        assert np.max(np.abs(P2[big] / P1[big] - 1.0)) < 1e-12


def test_zero_field_gives_ground_state(c1):
    # pruning appendix: no non-zero heating term -> P_i = delta_i0
    w, u, s = c1
    P, j = oracle.solve_pair(np.zeros_like(u[0]), w.grains[0], w.lam_cm)
    assert P[0] == 1.0 and np.all(P[1:] == 0.0)
    assert np.allclose(j, s.cabs * s.planck[0], rtol=1e-15, atol=0)


def test_loglog_interpolation_exact_on_power_laws(c1):
    # with u C a power law in lambda, the interpolated heating rate equals the
    # closed form Omega(lambda_fi) lambda_fi^3 dE_f / (h^2 c) everywhere on the grid
    w, u, s = c1
    lam = w.lam_cm
    q = 1.3
    u_pl = 1e-9 * (lam / 1e-4) ** q / s.cabs          # u * C = 1e-9 (lambda / 1 um)^q
    A = om.heating_matrix(u_pl, s, intrabin=False)
    E, dE = s.E, s.dE
    n = E.shape[0]
    f, i = np.tril_indices(n, k=-1)
    lf = HC / (E[f] - E[i])
    inside = (lf >= lam[0]) & (lf <= lam[-1])
    ref = np.where(inside, 1e-9 * (lf / 1e-4) ** q * lf ** 3 * dE[f] / (H * H * C), 0.0)
    got = A[f, i]
    assert np.all((got == 0) == (ref == 0))
    nz = ref > 0
    assert np.max(np.abs(got[nz] / ref[nz] - 1.0)) < 1e-12


def test_heating_rate_counts_photons(c1):
    # A_fi equals the photon absorption rate into bin f: c u_E C dE_f / eps with
    # u_E = u_lambda lambda^2 / (h c) the energy density per unit photon energy.
    # Checked where lambda_fi falls exactly on a grid node (no interpolation).
    w, u, s = c1
    lam = w.lam_cm
    E, dE = s.E, s.dE
    # construct a pair (f, i) with lambda_fi = lam[123] by moving E_i
    f = 200
    target = lam[123]
    eps = HC / target
    Ei = E[f] - eps
    s2 = om.GrainSetup(lam=lam, cabs=s.cabs, longwave_index=s.longwave_index,
                       E=np.array([Ei, E[f]]), dE=np.array([dE[0], dE[f]]), T=s.T[:2], cool=s.cool[:2],
                       planck=s.planck[:2])
    A = om.heating_matrix(u[3], s2, intrabin=False)
    uE = u[3][123] * target ** 2 / HC
    photons = C * uE * s.cabs[123] * dE[f] / eps
    assert abs(A[1, 0] / photons - 1.0) < 1e-12


def test_energy_balance_c1(c1):
    w, u, s = c1
    for c in (0, 17, 40, 63):
        P, j, d = oracle.solve_pair(u[c], w.grains[0], w.lam_cm, with_diag=True)
        # (i) discrete heating power = discrete cooling power in the steady state
        assert abs(d["heat"] / d["cool"] - 1.0) < 1e-12
        # (ii) emission on the grid vs cooling power: differs only by emission beyond the grid
        assert abs(d["emitted"] / d["cool"] - 1.0) < 1e-3
        # (iii) emission vs the representable absorbed power
        assert abs(d["emitted"] / d["A_rep"] - 1.0) < 1e-2


def test_emission_cutoff(c1):
    # eq:emission-lambda: Lambda = 0 when E_i < h nu; no bin reaches 13.8 eV here
    # when E_max = 10 eV, so the shortest wavelengths carry no emission
    w, u, s = c1
    P, j = oracle.solve_pair(u[5], w.grains[0], w.lam_cm)
    cut = HC / w.lam_cm > s.E[-1]
    assert np.any(cut) and np.all(j[cut] == 0.0) and np.all(j[~cut] >= 0.0)


def test_large_grain_collapses_to_equilibrium_and_needs_intrabin():
    # a 250 A grain with 128 bins: P collapses to a narrow peak at T_eq.  The
    # paper-literal rates (no continuous intrabin term) miss the energy budget.
    lam = synth.wavelength_grid_cm(500)
    g = synth.make_grain("carbonaceous", 250e-8, lam)
    assert g.n_bins == 128
    s = oracle.grain_setup(g, lam)
    for U in (0.1, 1.0, 1e3, 1e5):
        u = make_fields(lam, FieldRecipe(5, (U, U), 0.0, None), 1)[0]
        P, j, d = oracle.solve_pair(u, g, lam, with_diag=True)
        Teq = oracle.equilibrium_temperature(u, s)
        k = int(np.argmax(P))
        width = s.T[k + 1] - s.T[k]
        Tmean = float(np.sum(P * s.T))
        Tsd = float(np.sqrt(np.sum(P * (s.T - Tmean) ** 2)))
        # the peak sits within 1.5 bins of T_eq, and its width is the few-bin
        # random walk that 128 bins allow (P_i ratio per bin ~ (T_i+1/T_i)^(4+p))
        assert abs(Tmean - Teq) <= 1.5 * width and abs(s.T[k] - Teq) <= 1.5 * width
        assert Tsd / Tmean < 0.12
        assert abs(d["emitted"] / d["absorbed"] - 1.0) < 0.01
        P0, j0, d0 = oracle.solve_pair(u, g, lam, intrabin=False, with_diag=True)
        assert d0["emitted"] / d0["absorbed"] < 0.5


def test_small_grain_is_stochastic():
    # a 3.5 A grain: broad P spanning many decades, still in energy balance
    lam = synth.wavelength_grid_cm(500)
    g = synth.make_grain("carbonaceous", 3.5e-8, lam)
    assert g.n_bins == 1024
    u = make_fields(lam, FieldRecipe(5, (1.0, 1.0), 0.0, None), 1)[0]
    P, j, d = oracle.solve_pair(u, g, lam, with_diag=True)
    assert abs(d["emitted"] / d["A_rep"] - 1.0) < 0.01
    assert P.max() < 0.1 and np.count_nonzero(P > 1e-3) > 50


def test_uneven_workload_grid_reaches_below_coldest_equilibrium():
    # The uneven workload's weakest field (U = 0.1 under tau_V = 20) cools the
    # largest grains further than any other workload's; the enthalpy grid must
    # start below that equilibrium temperature, else probability piles up in
    # the lowest bin and the grain emits more than it absorbs.
    w = synth.workload("c3_uneven", n_cells=1)
    rec = synth.FieldRecipe(seed=1, U_range=(0.1, 0.1 * (1 + 1e-9)), jitter=0.0,
                            tau_V_range=(20.0, 20.0 * (1 + 1e-9)))
    u = synth.fields.make_fields(w.lam_cm, rec, 1)[0]
    for gi in (63, 127):
        s = oracle.grain_setup(w.grains[gi], w.lam_cm)
        T_eq = oracle.equilibrium_temperature(u, s)
        assert T_eq > 1.5 * s.T[0], (gi, T_eq, s.T[0])
        P, _, d = oracle.solve_pair(u, w.grains[gi], w.lam_cm, with_diag=True)
        assert P[0] < 1e-3
        # below 6 K a sizeable part of the emission falls beyond 1000 um, off
        # the grid, so emitted-on-grid / absorbed sits below 1
        assert 0.8 < d["emitted"] / d["A_rep"] < 1.01


def test_size_convolution_is_the_weighted_sum():
    # eq:convolution on a discrete grid: linear in the weights, one unit
    # weight returns that grain's spectrum (times lambda when weighted)
    rng = np.random.default_rng(4)
    lam = synth.wavelength_grid_cm(50)
    j = rng.random((3, 4, 50))
    e = np.zeros(4)
    e[2] = 1.0
    assert np.array_equal(oracle.size_convolution(j, e, lam, lambda_weighted=False), j[:, 2])
    assert np.allclose(oracle.size_convolution(j, e, lam), j[:, 2] * lam, rtol=1e-15)
    w1, w2 = rng.random(4), rng.random(4)
    assert np.allclose(oracle.size_convolution(j, w1 + 2 * w2, lam),
                       oracle.size_convolution(j, w1, lam) + 2 * oracle.size_convolution(j, w2, lam), rtol=1e-13)


def test_power_law_size_weights_integrate_the_distribution():
    # sum_g w_g f(a_g) approximates int K a^-q f(a) da: with f = 1 the closed
    # form K (a_min^(1-q) - a_max^(1-q)) / (q - 1), to the midpoint rule's error
    r = synth.radii_cm(3.5, 250.0, 256)
    w = synth.size_weights(r, q=3.5, per_H=1.0)
    exact = (r[0] ** -2.5 - r[-1] ** -2.5) / 2.5
    assert abs(w.sum() / exact - 1) < 2e-3


def test_coarse_bin_energy_balance_across_the_batched_radii():
    # The batched workload's 14..48 A grains (528..288 bins) at strong fields:
    # the steady state balances exactly (discrete heating = cooling), the
    # spectrum carries the cooling power, and yet emitted / A_rep ranges over
    # about 0.92..1.04.  The whole difference sits in the heating rates'
    # photon-energy sum: for one lower bin i the discrete heating power
    # H_i = sum_f A_fi (E_f - E_i) is a sum over the upper bins' photon energies
    # with weights dE_f (eq:heating), a quadrature of the absorbed power per
    # unit photon energy with nodes several eV apart once the bins are that
    # wide; where the field's power ends at the grid's short end (13.8 eV) such
    # a sum miscounts by up to half a node spacing times the power there.
    # It goes away as the bins are refined.
    w = synth.workload("c2_batched", n_cells=1)
    lam = w.lam_cm
    radii = synth.radii_cm(3.5, 250.0, 32)
    ratios = []
    for ai in range(10, 20):
        g = synth.make_grain("carbonaceous", radii[ai], lam)
        s = oracle.grain_setup(g, lam)
        for U in (1e3, 2e4, 1e5):
            u = make_fields(lam, FieldRecipe(1, (U, U), 0.0, None), 1)[0]
            A = om.heating_matrix(u, s)
            P, _, _ = om.recursion(om.b_matrix_recurrence(A), s.cool)
            j = om.emission(P, s)
            d = om.diagnostics(u, s, P, j, A)
            assert abs(d["heat"] / d["cool"] - 1.0) < 1e-12
            assert abs(d["emitted"] / d["cool"] - 1.0) < 1e-3
            assert abs(d["A_rep"] / d["absorbed"] - 1.0) < 1e-6
            # per lower bin: discrete heating power vs representable absorbed power
            dEm = s.E[:, None] - s.E[None, :]
            H = np.sum(A * np.where(dEm > 0, dEm, 0.0), axis=0)
            cum = om.absorbed_cumulative(u, s)
            edge = s.E[-1] + 0.5 * s.dE[-1] - s.E
            jrep = np.searchsorted(lam, HC / edge, side="left")
            R = np.append(cum, 0.0)[np.minimum(jrep, lam.shape[0])]
            quad = float(np.sum(P * H) / np.sum(P * R))
            ratio = d["emitted"] / d["A_rep"]
            assert abs(ratio / quad - 1.0) < 1e-3
            # bins far narrower than the field's photon energies hold no such error
            spacing = np.append(np.diff(s.E), np.inf)
            fine = (spacing < 0.05 * oracle.EV) & (R > 0)
            if np.any(fine):
                assert np.max(np.abs(H[fine] / R[fine] - 1.0)) < 0.01
            ratios.append(ratio)
    ratios = np.array(ratios)
    assert ratios.min() < 0.95 and ratios.max() > 1.01          # the imbalance is real on these bins
    assert 0.9 < ratios.min() and ratios.max() < 1.05
    # refinement: the 18.3 A grain at U = 2e4, 464 -> 1856 bins
    u = make_fields(lam, FieldRecipe(1, (2e4, 2e4), 0.0, None), 1)[0]
    out = []
    for n in (464, 1856):
        g = synth.make_grain("carbonaceous", radii[12], lam, n_bins=n)
        _, _, d = oracle.solve_pair(u, g, lam, with_diag=True)
        out.append(d["emitted"] / d["A_rep"])
    assert abs(out[0] - 1.0) > 0.02 and abs(out[1] - 1.0) < 1e-3


def test_table_method_twin():
    # the oracle's table method: exact at its nodes, exact for spectra that
    # are power laws in U between nodes, clamped outside the node range, and
    # without emission where a node it draws on has none
    from oracle import table as otab
    lam = synth.wavelength_grid_cm(400)
    g = synth.make_grain("carbonaceous", 20e-8, lam, n_bins=128)
    u_ref = make_fields(lam, FieldRecipe(0, (1.0, 1.0), 0.0, None), 1)[0]
    lo, hi, K = -1.0, 3.0, 5
    y = otab.build_table(g, lam, u_ref, lo, hi, K)
    x = otab.node_log10U(lo, hi, K)
    for k in (0, 2, 4):
        u = 10.0 ** x[k] * u_ref
        got = otab.lookup(y, lo, hi, u, u_ref, g.cabs_cm2, lam)
        _, j = oracle.solve_pair(u, g, lam)
        m = j > 0
        assert np.all(got[~m] == 0.0) and np.allclose(got[m], j[m], rtol=1e-12, atol=0)
    # a synthetic table that is a power law in U: j / A = 2^c U^p
    rng = np.random.default_rng(3)
    c = rng.normal(-20, 3, lam.shape[0])
    p = 0.7
    ypl = c[None, :] + p * np.log2(10.0 ** x)[:, None]
    for U in (0.37, 1.0, 55.5, 999.0):
        u = U * u_ref
        A = otab.absorbed_power(u, g.cabs_cm2, lam)
        got = otab.lookup(ypl, lo, hi, u, u_ref, g.cabs_cm2, lam)
        assert np.allclose(got, A * 2.0 ** c * U ** p, rtol=1e-12)
    # clamped: a field weaker than the first node takes that node's shape
    u = 1e-3 * u_ref
    got = otab.lookup(ypl, lo, hi, u, u_ref, g.cabs_cm2, lam)
    assert np.allclose(got, otab.absorbed_power(u, g.cabs_cm2, lam) * 2.0 ** c * 0.1 ** p, rtol=1e-12)
    # a node without emission at one wavelength: none between it and the next node
    yz = ypl.copy()
    yz[1, 7] = -np.inf
    got = otab.lookup(yz, lo, hi, 3.0 * u_ref, u_ref, g.cabs_cm2, lam)      # between nodes 1 and 2
    assert got[7] == 0.0 and got[8] > 0.0
    got = otab.lookup(yz, lo, hi, 100.0 * u_ref, u_ref, g.cabs_cm2, lam)    # exactly node 3 (w = 0)
    assert got[7] > 0.0
    # the table's energy budget: node k's ratio times its absorbed power is
    # the emitted power of that node's solve, as the oracle's diagnostics
    # integrate it
    rho = otab.node_ratios(y, lam)
    for k in (0, 2, 4):
        u = 10.0 ** x[k] * u_ref
        _, _, d = oracle.solve_pair(u, g, lam, with_diag=True)
        A = otab.absorbed_power(u, g.cabs_cm2, lam)
        assert abs(rho[k] * A / d["emitted"] - 1.0) < 1e-12
        # and the interpolated budget at a node is that node's ratio
        assert otab.budget_ratio(rho, lo, hi, u, u_ref, lam) == pytest.approx(rho[k], rel=1e-14)


def test_table_budget_closed_forms():
    # node_ratios: 4 pi int 2^y dlambda, exact for spectra linear in lambda
    # (the trapezoid rule), a node value without emission contributing nothing;
    # budget_ratio: linear in the node coordinate, clamped at both ends
    from oracle import table as otab
    lam = synth.wavelength_grid_cm(300)
    l0, l1 = lam[0], lam[-1]
    K = 4
    a = np.array([1.0, 2.0, 0.5, 3.0])
    b = np.array([0.0, 1e3, -4.0, 5e2])           # a + b lambda > 0 on the grid
    y = np.log2(a[:, None] + b[:, None] * lam[None, :])
    rho = otab.node_ratios(y, lam)
    exact = 4 * math.pi * (a * (l1 - l0) + 0.5 * b * (l1 ** 2 - l0 ** 2))
    assert np.allclose(rho, exact, rtol=1e-12)
    yz = np.zeros((1, lam.shape[0]))
    yz[0, 5] = -np.inf                    # j / A = 1 except at node 5
    w5 = 0.5 * (lam[6] - lam[4])
    assert otab.node_ratios(yz, lam)[0] == pytest.approx(4 * math.pi * (l1 - l0 - w5), rel=1e-13)
    lo, hi = 0.0, 3.0
    u_ref = np.ones_like(lam)
    x = otab.node_log10U(lo, hi, K)
    for k in range(K):
        assert otab.budget_ratio(rho, lo, hi, 10.0 ** x[k] * u_ref, u_ref, lam) == pytest.approx(rho[k], rel=1e-14)
    mid = 10.0 ** (0.5 * (x[1] + x[2]))
    assert otab.budget_ratio(rho, lo, hi, mid * u_ref, u_ref, lam) == pytest.approx(0.5 * (rho[1] + rho[2]), rel=1e-12)
    assert otab.budget_ratio(rho, lo, hi, 1e-3 * u_ref, u_ref, lam) == pytest.approx(rho[0], rel=1e-14)
    assert otab.budget_ratio(rho, lo, hi, 1e6 * u_ref, u_ref, lam) == pytest.approx(rho[-1], rel=1e-14)
