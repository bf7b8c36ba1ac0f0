"""Pins of the oracle's system matrix (Siddon intersection lengths) and projector pair."""
import numpy as np
import pytest

import oracle


def clip_length(c, s, u, X0, X1, Y0, Y1):
    """Length of the line x c + y s = u inside the rectangle [X0,X1]x[Y0,Y1] (Liang-Barsky)."""
    px, py = u * c, u * s  # foot point
    dx, dy = -s, c
    t0, t1 = -1e300, 1e300
    for p, q in ((-dx, px - X0), (dx, X1 - px), (-dy, py - Y0), (dy, Y1 - py)):
        if p == 0.0:
            if q < 0:
                return 0.0
        else:
            t = q / p
            if p < 0:
                t0 = max(t0, t)
            else:
                t1 = min(t1, t)
    return max(0.0, t1 - t0)


def chord(c, s, h, t):
    """Chord of a line at signed distance t from the centre of an h-square (closed square)."""
    ac, as_ = abs(c), abs(s)
    w1 = 0.5 * h * (ac + as_)
    w0 = 0.5 * h * abs(ac - as_)
    m = h / max(ac, as_)
    at = abs(t)
    if at <= w0:
        return m
    if at >= w1:
        return 0.0
    return m * (w1 - at) / (w1 - w0)


def test_axis_aligned_rays_through_pixel_centres():
    g = oracle.Geometry(16, 12, 1, 2.0, 4, 16, 2.0)
    A = oracle.system_matrix(g).toarray()
    # angle 0: normal (1, 0) -> vertical lines x = u_b through column b's centres
    for b in range(16):
        row = A[0 * 16 + b].reshape(12, 16)
        np.testing.assert_allclose(row[:, b], 2.0, rtol=1e-13)
        assert np.count_nonzero(row) == 12
    # angle 2 (90 deg): horizontal lines y = u_b; bins beyond the 12 rows miss the image
    for b in range(16):
        row = A[2 * 16 + b].reshape(12, 16)
        yb = (b - 7.5) * 2.0
        j = int(np.floor((yb + 12.0) / 2.0))
        if 0 <= j < 12:
            np.testing.assert_allclose(row[j], 2.0, rtol=1e-13)
            assert np.count_nonzero(row) == 16
        else:
            assert np.count_nonzero(row) == 0


def test_diagonal_ray_through_corners():
    g = oracle.Geometry(8, 8, 1, 1.5, 4, 8, 1.5)
    idx, ln = oracle.siddon_line(g, np.sqrt(0.5), np.sqrt(0.5), 0.0)  # x + y = 0: anti-diagonal
    assert len(idx) == 8
    np.testing.assert_allclose(ln, 1.5 * np.sqrt(2.0), rtol=1e-14)
    j, i = np.divmod(idx, 8)
    assert np.all(i + j == 7)


def test_half_open_tie_rule():
    g = oracle.Geometry(4, 4, 1, 1.0, 2, 4, 1.0)
    idx, ln = oracle.siddon_line(g, 1.0, 0.0, 0.0)  # x = 0 is the boundary between columns 1 and 2
    assert np.all(idx % 4 == 2) and np.allclose(ln, 1.0)
    idx, _ = oracle.siddon_line(g, 1.0, 0.0, 2.0)  # right image edge: outside (half-open)
    assert len(idx) == 0
    idx, _ = oracle.siddon_line(g, 1.0, 0.0, -2.0)  # left edge belongs to column 0
    assert np.all(idx % 4 == 0)


def test_ray_sum_equals_clipped_length_and_square_chords():
    rng = np.random.default_rng(3)
    for trial in range(200):
        nx, ny = rng.integers(3, 24, 2)
        h = rng.uniform(0.5, 3.0)
        th = rng.uniform(0, np.pi)
        c, s = np.cos(th), np.sin(th)
        u = rng.uniform(-0.6, 0.6) * h * max(nx, ny)
        g = oracle.Geometry(int(nx), int(ny), 1, h, 1, 1, h)
        idx, ln = oracle.siddon_line(g, c, s, u)
        X0, Y0 = -nx * h / 2, -ny * h / 2
        total = clip_length(c, s, u, X0, -X0, Y0, -Y0)
        assert ln.sum() == pytest.approx(total, rel=1e-12, abs=1e-12)
        dense = np.zeros(nx * ny)
        np.add.at(dense, idx, ln)
        xc = (np.arange(nx) - (nx - 1) / 2) * h
        yc = (np.arange(ny) - (ny - 1) / 2) * h
        ref = np.array([chord(c, s, h, u - xc[i] * c - yc[j] * s) for j in range(ny) for i in range(nx)])
        np.testing.assert_allclose(dense, ref, rtol=0, atol=1e-11 * h)


def test_lengths_against_brute_force_clipping_per_pixel():
    g = oracle.Geometry(7, 5, 1, 1.3, 9, 11, 0.9, ang0=0.1)
    A = oracle.system_matrix(g).toarray()
    for a in range(9):
        c, s = g.cos_sin(a)
        for b in range(11):
            u = g.bin_centre(b)
            for j in range(5):
                for i in range(7):
                    X0 = -3.5 * 1.3 + i * 1.3
                    Y0 = -2.5 * 1.3 + j * 1.3
                    ref = clip_length(c, s, float(u), X0, X0 + 1.3, Y0, Y0 + 1.3)
                    assert A[a * 11 + b, j * 7 + i] == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("Q", [1, 4, 7])
def test_adjointness_and_subset_partition(Q):
    g = oracle.Geometry(24, 20, 3, 2.0, 30, 26, 1.7)
    rng = np.random.default_rng(Q)
    x = rng.random((3, 20, 24, 5))
    full = oracle.forward(g, x)
    for q in range(Q):
        y = rng.random((3, len(oracle.subset_angles(30, q, Q)), 26, 5))
        fx = oracle.forward(g, x, q, Q)
        bty = oracle.back(g, y, q, Q)
        lhs, rhs = np.sum(fx * y), np.sum(x * bty)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        np.testing.assert_array_equal(fx, full[:, oracle.subset_angles(30, q, Q)])
        ones = np.ones_like(y[..., :1])
        np.testing.assert_allclose(oracle.back(g, ones, q, Q)[0, :, :, 0], oracle.subset_sensitivity(g, q, Q),
                                   rtol=1e-14)
    # planes are independent: each plane is the 2D projection of its own slice
    np.testing.assert_allclose(full[1], oracle.forward(g, x[1:2])[0], rtol=1e-15)
