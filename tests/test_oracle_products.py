"""CPU pins of the difference-image products oracle (multi-template median
combine, aperture photometry, limiting magnitude) against definitions that
do not share its code: a sort-based median in pure Python, known magnitude
differences, sub-pixel grid counts, the disk area, hand-computed cases."""
import math

import numpy as np
import pytest

from oracle import products as P


def _py_median(vals):
    v = sorted(vals)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
def test_median_combine_matches_sorted_middle(n):
    rng = np.random.default_rng(10 + n)
    diffs = [rng.normal(size=(5, 6)) for _ in range(n)]
    zps = list(rng.uniform(24, 27, size=n))
    out = P.median_combine(diffs, zps, 25.0)
    for y in range(5):
        for x in range(6):
            vals = [diffs[t][y, x] * 10 ** (0.4 * (25.0 - zps[t])) for t in range(n)]
            assert out[y, x] == pytest.approx(_py_median(vals), rel=1e-14, abs=1e-15)


def test_zero_point_scale_known_values():
    # 2.5 magnitudes is a factor 10; 5 magnitudes 100; equal zero points 1
    assert P.zp_scale(25.0, 27.5) == pytest.approx(10.0, rel=1e-15)
    assert P.zp_scale(30.0, 25.0) == pytest.approx(0.01, rel=1e-15)
    assert P.zp_scale(26.3, 26.3) == 1.0
    # a source of magnitude m keeps it: zp_to - 2.5 log10(f * scale) == zp_from - 2.5 log10(f)
    f = 1234.5
    assert 27.0 - 2.5 * math.log10(f * P.zp_scale(25.2, 27.0)) == pytest.approx(25.2 - 2.5 * math.log10(f))


def test_median_of_identical_stack_is_the_image():
    rng = np.random.default_rng(3)
    D = rng.normal(size=(8, 8))
    out = P.median_combine([D] * 5, [25.0] * 5, 25.0)
    assert np.array_equal(out, D)


def test_median_rejects_one_outlier_template():
    # four agreeing differences and one with a large artefact: the median
    # is the agreeing value wherever the artefact sits
    D = np.full((4, 4), 2.0)
    bad = D.copy()
    bad[1, 2] = 1e6
    out = P.median_combine([D, D, bad, D, D], [25.0] * 5, 25.0)
    assert np.array_equal(out, D)


def _grid_area(cx, cy, r, px, py, n=1200):
    # midpoint sub-pixel count on an n x n grid
    t = (np.arange(n) + 0.5) / n - 0.5
    X = px + t[None, :] - cx
    Y = py + t[:, None] - cy
    return float(np.count_nonzero(X * X + Y * Y <= r * r)) / (n * n)


@pytest.mark.parametrize("cx,cy,r,px,py", [
    (10.0, 10.0, 3.0, 10, 10), (10.0, 10.0, 3.0, 12, 11), (10.0, 10.0, 3.0, 13, 10),
    (10.3, 9.71, 2.5, 12, 8), (5.5, 5.5, 0.4, 5, 5), (5.5, 5.5, 0.4, 6, 6), (7.25, 3.8, 4.1, 10, 1),
])
def test_overlap_area_matches_subpixel_count(cx, cy, r, px, py):
    a = P.overlap_area(cx, cy, r, px, py)
    g = _grid_area(cx, cy, r, px, py)
    # the grid count has an O(perimeter / n) error
    assert abs(a - g) <= 3.0 / 1200
    assert 0.0 <= a <= 1.0


def test_overlap_area_full_and_empty_pixels():
    assert P.overlap_area(10.0, 10.0, 3.0, 10, 10) == pytest.approx(1.0, abs=1e-14)
    assert P.overlap_area(10.0, 10.0, 3.0, 14, 10) == 0.0
    # a pixel wholly inside a large circle
    assert P.overlap_area(0.0, 0.0, 10.0, 3, 4) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("cx,cy,r", [(20.0, 20.0, 3.0), (20.37, 19.62, 3.0), (15.5, 16.25, 5.7), (12.1, 12.9, 0.8)])
def test_aperture_weights_sum_to_disk_area(cx, cy, r):
    ys, xs, w = P.aperture_weights(cx, cy, r, 64, 64)
    assert float(np.sum(w)) == pytest.approx(math.pi * r * r, rel=1e-11)


def test_aperture_flux_of_constant_and_edge_cut():
    img = np.full((40, 50), 3.0)
    f = P.aperture_flux(img, [(25.0, 20.0), (25.4, 19.3)], 3.0)
    assert np.allclose(f, 3.0 * math.pi * 9.0, rtol=1e-11)
    # centred on the corner pixel: the image keeps x, y >= -1/2 of the disk,
    # a quarter disk, two strips of width 1/2 along the axes and the
    # [-1/2, 0]^2 square; strip = integral_0^(1/2) sqrt(9 - u^2) du
    strip = 0.5 * (0.5 * math.sqrt(9 - 0.25) + 9 * math.asin(0.5 / 3))
    fc = P.aperture_flux(img, [(0.0, 0.0)], 3.0)[0]
    assert fc == pytest.approx(3.0 * (math.pi * 9.0 / 4 + 2 * strip + 0.25), rel=1e-11)


def test_aperture_flux_point_source():
    # a single bright pixel inside the aperture gives its value times its area
    img = np.zeros((30, 30))
    img[12, 14] = 100.0
    f = P.aperture_flux(img, [(14.0, 12.0), (14.5, 12.0), (20.0, 20.0)], 2.0)
    assert f[0] == pytest.approx(100.0, rel=1e-13)
    assert f[1] == pytest.approx(100.0 * P.overlap_area(14.5, 12.0, 2.0, 14, 12), rel=1e-13)
    assert f[2] == 0.0


def test_limiting_magnitude_hand_case():
    # four apertures on an image that is +1 / -1 per half: fluxes known,
    # sample std by hand, m_lim = zp - 2.5 log10(5 sigma)
    img = np.zeros((40, 40))
    img[:, :20] = 1.0
    img[:, 20:] = -1.0
    xy = [(8.0, 10.0), (8.0, 30.0), (31.0, 10.0), (31.0, 30.0)]
    sigma, mlim, f = P.limiting_magnitude(img, xy, 3.0, 30.0)
    A = math.pi * 9.0
    assert np.allclose(f, [A, A, -A, -A], rtol=1e-11)
    s = math.sqrt(4 * A * A / 3)
    assert sigma == pytest.approx(s, rel=1e-11)
    assert mlim == pytest.approx(30.0 - 2.5 * math.log10(5 * s), rel=1e-12)


def test_forced_photometry_magnitudes():
    img = np.zeros((30, 30))
    img[10, 10] = 1000.0
    img[20, 20] = -50.0
    f, m, e = P.forced_photometry(img, [(10.0, 10.0), (20.0, 20.0)], 1.0, 28.0, 5.0)
    assert f[0] == pytest.approx(1000.0, rel=1e-12)
    assert m[0] == pytest.approx(28.0 - 7.5, abs=1e-12)
    assert e[0] == pytest.approx(2.5 / math.log(10) * 5.0 / 1000.0, rel=1e-12)
    assert math.isnan(m[1]) and e[1] == pytest.approx(2.5 / math.log(10) * 5.0 / 50.0, rel=1e-12)
