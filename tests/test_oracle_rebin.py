"""Pins of the rebinning oracle against what the definition fixes: where one ring pair's sinogram
lands, conservation of counts, the number of ring pairs per plane in closed form, and that the
entries of ring pairs outside the scanner are never read."""
import numpy as np
import pytest

import oracle


def test_one_ring_pair_lands_on_plane_r1_plus_r2():
    R, D = 6, 3
    for r1, r2 in [(0, 0), (2, 5), (5, 2), (4, 1), (5, 5)]:
        y = np.zeros((2 * D + 1, R, 2, 3, 1))
        y[r2 - r1 + D, r1, 1, 2, 0] = 7.0
        out, _ = oracle.ssrb(y, R, D)
        z, a, b, m = np.nonzero(out)
        assert list(z) == [r1 + r2] and out[r1 + r2, 1, 2, 0] == 7.0


@pytest.mark.parametrize("R,D", [(1, 0), (4, 0), (5, 2), (8, 7)])
def test_counts_conserved_and_pairs_per_plane(R, D):
    rng = np.random.default_rng(R * 10 + D)
    y = rng.poisson(3.0, (2 * D + 1, R, 3, 4, 2)).astype(float)
    # entries whose ring pair does not exist: first ring r1 with r1 + delta outside [0, R)
    valid = np.zeros((2 * D + 1, R), dtype=bool)
    for d in range(2 * D + 1):
        for r1 in range(R):
            valid[d, r1] = 0 <= r1 + d - D < R
    y[~valid] = np.nan  # must never be read
    out, count = oracle.ssrb(y, R, D)
    assert np.all(np.isfinite(out))
    assert out.sum() == pytest.approx(np.nansum(y))
    z = np.arange(2 * R - 1)
    # pairs (r1, r2) with r1 + r2 = z, both in [0, R) and |r2 - r1| = |z - 2 r1| <= D
    closed = np.array([sum(1 for r1 in range(R) if 0 <= zz - r1 < R and abs(zz - 2 * r1) <= D) for zz in z])
    assert np.array_equal(count, closed)
    if D == R - 1:  # every pair: min(z, 2R - 2 - z) + 1
        assert np.array_equal(count, np.minimum(z, 2 * R - 2 - z) + 1)
    if D == 0:  # direct planes only
        assert np.array_equal(count, (z % 2 == 0).astype(float))
