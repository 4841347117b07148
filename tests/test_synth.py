"""Seeded synthetic inputs: shapes, conventions and the field normalisation
pinned to the paper's ISRF energy density (CPU only)."""

import json
import math
import os

import numpy as np

import synth
from synth.fields import make_fields, FieldRecipe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_field_energy_density_matches_paper_isrf():
    ref = json.load(open(GOLDEN))["isrf_energy_density_eV_cm3"]
    lam = np.geomspace(1e-7, 1e2, 40001)
    u = make_fields(lam, FieldRecipe(1, (1.0, 1.0), 0.0, None), 1)[0]
    total = np.trapezoid(u, lam) / synth.CONSTANTS["eV"]
    assert round(total, ref["digits"]) == ref["value"]
    assert abs(total - 0.46268) < 1e-4
    grid = synth.wavelength_grid_cm(500)
    ug = make_fields(grid, FieldRecipe(1, (1.0, 1.0), 0.0, None), 1)[0]
    assert abs(np.trapezoid(ug, grid) / synth.CONSTANTS["eV"] - 0.4597) < 2e-4


def test_wavelength_grid():
    lam = synth.wavelength_grid_cm(500)
    assert lam[0] == 0.09e-4 and abs(lam[-1] / 0.1 - 1) < 1e-15
    r = lam[1:] / lam[:-1]
    assert np.allclose(r, r[0], rtol=1e-13, atol=0)


def test_bin_law_and_shapes():
    w2 = synth.workload("c2_batched", n_cells=4)
    bins = [g.n_bins for g in w2.grains]
    assert bins[0] == 1024 and bins[-1] == 128 and sum(bins) == 13968
    assert all(b % 16 == 0 for b in bins)
    w3 = synth.workload("c3_uneven", n_cells=4)
    assert len(w3.grains) == 128 and sum(g.n_bins for g in w3.grains) == 2 * 21056
    w1 = synth.workload("c1_tiny")
    assert w1.n_pairs == 64 and w1.grains[0].n_bins == 256 and w1.n_lambda == 400


def test_seeded_prefix_and_ranges():
    w = synth.workload("c2_batched")
    a = make_fields(w.lam_cm, w.field_recipe, w.n_cells, cells=np.arange(5))
    b = make_fields(w.lam_cm, w.field_recipe, w.n_cells, cells=np.arange(3))
    assert np.array_equal(a[:3], b)
    from synth.fields import field_parameters
    U, jit, tau = field_parameters(w.field_recipe, w.n_cells)
    assert U.min() >= 0.1 and U.max() <= 1e5 and jit.min() >= 0.7 and jit.max() <= 1.3
    w3 = synth.workload("c3_uneven")
    U3, _, tau3 = field_parameters(w3.field_recipe, w3.n_cells)
    assert tau3.min() >= 0.01 and tau3.max() <= 20.0 and U3.max() <= 1e3
    u3 = make_fields(w3.lam_cm, w3.field_recipe, w3.n_cells, cells=np.arange(8))
    assert np.all(np.isfinite(u3)) and np.all(u3 > 0)
