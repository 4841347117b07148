"""Host logic of the benchmark: how the surrogate's radius ranges are formed,
the error measures it reports (band errors, relative error of j against the
oracle), its roofline accounting, and when it reports the recorded HBM
traffic."""

import numpy as np

import bench
import synth


def test_radius_groups_partition_each_composition_in_order():
    w = synth.workload("c4_train")
    for comp in ("carbonaceous", "silicate"):
        groups = bench.radius_groups(w.grains, comp, 4)
        assert len(groups) == 4
        idx = [i for g in groups for i, _ in g]
        mine = [i for i, g in enumerate(w.grains) if g.composition == comp]
        assert idx == mine                                   # every grain once, in order
        assert all(len(g) == len(mine) // 4 for g in groups)
        for g in groups:
            assert all(gr.composition == comp for _, gr in g)
            r = [gr.radius_cm for _, gr in g]
            assert r == sorted(r)
        # ranges do not overlap
        assert all(groups[k][-1][1].radius_cm < groups[k + 1][0][1].radius_cm for k in range(3))


def test_radius_groups_uneven_split_keeps_every_grain():
    w = synth.workload("c4_train")
    groups = bench.radius_groups(w.grains, "silicate", 5)
    sizes = [len(g) for g in groups]
    assert sum(sizes) == 64 and max(sizes) - min(sizes) <= 1


def test_band_error_uniform_scale_is_exact():
    lam = np.geomspace(1e-5, 1e-1, 500)
    rng = np.random.default_rng(1)
    jr = rng.uniform(0.5, 2.0, size=(3, 500))
    err = bench._band_error(1.05 * jr, jr, lam)
    assert np.allclose(err, 0.05, rtol=0, atol=1e-12)


def test_band_error_ignores_bands_without_power():
    lam = np.linspace(1.0, 2.0, 500)             # every band holds ~1/32 of a flat spectrum's power
    e1 = (1 * (500 - 1)) // 32                  # first node of band 1
    jr = np.ones((1, 500))
    jr[0, :e1 + 1] = 1e-12                       # band 0 holds ~1e-12 of the power
    jp = jr.copy()
    jp[0, :e1] *= 100.0                          # wrong by 99x, but only inside band 0
    assert bench._band_error(jp, jr, lam)[0] < 1e-12        # up to the rounding of the band sums
    jp[0, e1 + 2] *= 1.5                         # a change inside band 1 is seen
    assert bench._band_error(jp, jr, lam)[0] > 1e-3


def test_j_rel_err_masks_tiny_reference_values():
    jr = np.array([1.0, 0.5, 1e-12, 0.0])
    j = np.array([1.0 + 2e-5, 0.5 * (1 - 3e-5), 5e-12, 1.0])
    assert abs(bench.j_rel_err(j, jr) - 3e-5) < 1e-12
    assert bench.j_rel_err(np.zeros(3), np.zeros(3)) == 0.0
    assert bench.j_rel_err(np.ones(3), np.zeros(3)) == float("inf")


def test_roofline_accounting():
    # nine lane-cycles per on-grid rate against 256 CUs x 64 lanes x 2.4 GHz;
    # the exponential (one per rate) against half that lane rate
    r = bench.roofline(rates=4.0e10, solve_ms=40.0, traffic=None)
    assert r["bound"] == "alu" and r["peak"] == 256 * 64 * 2.4e9 / 1e12
    assert abs(r["achieved"] - 4.0e10 * 9 / 0.040 / 1e12) < 1e-9
    assert abs(r["frac"] - 4.0e10 * 9 / 0.040 / (256 * 64 * 2.4e9)) < 1e-12
    assert abs(r["exp2"]["frac"] - 4.0e10 / 0.040 / (256 * 64 * 2.4e9 / 2)) < 1e-12


def test_oracle_pairs_are_the_oracle_spectra():
    # the CPU leg's pool (setups handed to the solving workers) returns what
    # the oracle computes for each pair directly
    import oracle
    from synth.fields import make_fields
    w = synth.workload("c1_tiny")
    rec, spectra = bench.oracle_pairs("c1_tiny", w.n_cells, {0: [3, 40]})
    assert set(spectra) == {(3, 0), (40, 0)}
    u = make_fields(w.lam_cm, w.field_recipe, w.n_cells, cells=np.array([3, 40]))
    for k, c in enumerate((3, 40)):
        assert np.array_equal(spectra[(c, 0)], oracle.solve_pair(u[k], w.grains[0], w.lam_cm)[1])
    assert rec["kind"] == "oracle" and rec["value"] > 0 and rec["cores"] == bench.CPU_PROCS


def test_traffic_reported_only_for_the_recorded_solver_sources(tmp_path, monkeypatch):
    # the committed counter summary names the solver sources' hash; the bench
    # reports its bytes while the sources hash to it and null once they change
    import os
    import shutil
    for f in bench.SOLVER_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), tmp_path / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    summary = tmp_path / "profiles" / "solve_c5_hbm_traffic.md"
    summary.write_text("solve_phase_hbm_bytes_per_step: 1.5e+09\n"
                       f"solver_sources_sha256_16: {bench.solver_hash()}\n")
    assert bench.recorded_traffic("c5_surrogate") == 1.5e9
    assert bench.recorded_traffic("c2_batched") is None           # no summary for this workload
    with open(tmp_path / bench.SOLVER_SOURCES[0], "a") as fh:
        fh.write("\n")
    assert bench.recorded_traffic("c5_surrogate") is None
