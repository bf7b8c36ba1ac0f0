"""CPU: the comparison study's inputs and statistics (no device code)."""
import numpy as np
import pytest

from paper_1803_10045_amd import compare, inputs, kcs


def test_roi_stats_closed_form():
    truth = np.full((4, 5), 2.0)
    region = np.zeros((4, 5), dtype=bool)
    region[1:3, 1:4] = True
    a, e = 0.03, 0.05
    est = np.stack([truth * (1 + a + e), truth * (1 + a - e)])
    est[:, ~region] = 99.0  # outside the region: ignored
    st = compare.roi_stats(est, truth, region)
    assert st["bias_pct"] == pytest.approx(100 * a, rel=1e-12)
    assert st["std_pct"] == pytest.approx(100 * e * np.sqrt(2.0), rel=1e-12)


def test_ring_phantom_regions_and_table_values():
    cfg = inputs.rings_config(64, nz=2)
    lab = inputs.ring_labels(cfg)
    maps, obj = inputs.phantom_maps(cfg)
    assert lab.shape == (2, 64, 64) and set(np.unique(lab)) == {0, 1, 2, 3, 4}
    assert np.array_equal(obj, lab > 0)
    for reg, par in ((2, inputs.TABLE1_INNER), (3, inputs.TABLE1_MIDDLE), (4, inputs.TABLE1_OUTER)):
        for p in range(3):
            assert np.all(maps[p][lab == reg] == par[p])
    assert np.all(maps[0][lab == 1] == 0.0) and np.all(maps[1:, lab == 1] > 0.0) and np.all(maps[:, lab == 0] == 0.0)
    # rings nest outward: inner < middle < outer in mean radius
    yy, xx = np.meshgrid(np.arange(64) - 31.5, np.arange(64) - 31.5, indexing="ij")
    rad = [np.hypot(yy, xx)[lab[0] == r].mean() for r in (1, 2, 3, 4)]
    assert rad == sorted(rad)


def test_true_ki_and_method_priors():
    maps = np.array([[0.75, 0.0], [0.35, 0.0], [0.031, 0.0]]).reshape(3, 1, 2)
    ki = compare.true_ki(maps)
    assert ki[0, 0] == pytest.approx(0.75 * 0.031 / 0.381) and ki[0, 1] == 0.0
    base = kcs.Prior(0.1, 1e-3, 0.2, (1e-3,) * 3, True)
    ind, dire, kc = (compare.method_prior(base, m, 0.5) for m in compare.METHODS)
    assert (ind.kp_on, ind.beta_h) == (False, 0.0)
    assert (dire.kp_on, dire.beta_h) == (True, 0.0)
    assert (kc.kp_on, kc.beta_h) == (True, 0.5)
    with pytest.raises(ValueError):
        compare.method_prior(base, "osem", 0.1)
