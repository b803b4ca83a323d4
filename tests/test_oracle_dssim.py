"""Pins of the FP64 D-SSIM reference (Sec. 3.4, eq. 8; window, constants and border rule as
read in the reference's header): library routines, closed forms, invariants and finite
differences."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import dssim as D


def _rand(seed, shape):
    return np.random.default_rng(seed).uniform(0, 1, size=shape)


def test_window_sum_is_a_zero_filled_correlation():
    # an asymmetric kernel fixes the direction of the shift
    img = _rand(1, (9, 13))
    k = _rand(2, (11, 11))
    np.testing.assert_allclose(D.window_sum(img, k), correlate2d(img, k, mode="same", boundary="fill"), atol=1e-12)


def test_gaussian_window_closed_form():
    w = D.gaussian_window()
    r = np.arange(11) - 5.0
    g = np.exp(-r ** 2 / (2 * 1.5 ** 2))
    np.testing.assert_allclose(w, np.outer(g, g) / g.sum() ** 2, rtol=1e-14)
    assert abs(w.sum() - 1.0) < 1e-14 and np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])


def test_identical_images_have_zero_loss_and_gradient():
    x = _rand(3, (3, 14, 17))
    assert abs(D.dssim(x, x)) < 1e-14
    assert np.abs(D.dssim_grad(x, x)).max() < 1e-14


def test_constant_images_interior_closed_form():
    a, b = 0.3, 0.7
    x, y = np.full((24, 24), a), np.full((24, 24), b)
    s = D.ssim_terms(x, y, D.gaussian_window())[0]
    inner = s[5:-5, 5:-5]          # windows that stay inside the image
    np.testing.assert_allclose(inner, (2 * a * b + D.C1) / (a * a + b * b + D.C1), rtol=1e-12)
    # at the border the window sees zeros: the local means shrink, so SSIM differs there
    assert abs(s[0, 0] - inner[0, 0]) > 1e-6


def test_symmetric_and_bounded():
    x, y = _rand(4, (3, 12, 15)), _rand(5, (3, 12, 15))
    assert abs(D.dssim(x, y) - D.dssim(y, x)) < 1e-14
    assert 0.0 <= D.dssim(x, y) <= 2.0


@pytest.mark.parametrize("seed", [6, 7])
def test_gradient_matches_central_differences(seed):
    x, y = _rand(seed, (3, 9, 11)), _rand(seed + 10, (3, 9, 11))
    g = D.dssim_grad(x, y)
    h = 1e-6
    rng = np.random.default_rng(seed)
    for idx in [tuple(rng.integers(0, n) for n in x.shape) for _ in range(25)] + [(0, 0, 0), (2, 8, 10), (1, 4, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (D.dssim(xp, y) - D.dssim(xm, y)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-4), (idx, fd, g[idx])


def test_loss_matches_a_library_gaussian_filter():
    """The whole loss recomputed with SciPy's separable Gaussian filter (standard deviation 1.5,
    radius 5 via truncate, zero padding: the same window) and the SSIM formula."""
    from scipy.ndimage import gaussian_filter

    x, y = _rand(8, (3, 19, 23)), _rand(9, (3, 19, 23))
    f = lambda a: gaussian_filter(a, 1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
    tot = 0.0
    for ch in range(3):
        mx, my = f(x[ch]), f(y[ch])
        sxx, syy, sxy = f(x[ch] ** 2) - mx ** 2, f(y[ch] ** 2) - my ** 2, f(x[ch] * y[ch]) - mx * my
        s = (2 * mx * my + D.C1) * (2 * sxy + D.C2) / ((mx ** 2 + my ** 2 + D.C1) * (sxx + syy + D.C2))
        tot += s.sum()
    assert abs(D.dssim(x, y) - (1.0 - tot / x.size)) < 1e-12
