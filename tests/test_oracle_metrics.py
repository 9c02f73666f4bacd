"""Pins of the oracle's halftone metrics: the Gaussian windows, valid-mode
filtering against scipy's correlation, HVS-MSE special cases, and closed
forms of SSIM and of the contrast-weighted SSIM (CSSIM)."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from paper_2304_12152_amd import synth


def test_gauss_window_normalised_and_symmetric(orc):
    for sigma, r in ((2.0, 5), (1.5, 5), (1.0, 1)):
        g = orc.gauss_window(sigma, r)
        assert abs(g.sum() - 1.0) < 1e-15
        np.testing.assert_array_equal(g, g.T)
        np.testing.assert_array_equal(g, g[::-1, :])
        np.testing.assert_array_equal(g, g[:, ::-1])


def test_gauss_window_values(orc):
    # 11x11, sigma 2: the 1-D factor sums to 4.9859; centre 1/24.8592 and
    # corner exp(-6.25)/24.8592 (values computed by hand)
    g = orc.gauss_window(2.0, 5)
    assert abs(g[5, 5] - 0.0402265) < 5e-8
    assert abs(g[0, 0] - 7.766e-5) < 5e-9
    # separable: the window is the outer product of its normalised 1-D profile
    t = np.exp(-np.arange(-5, 6) ** 2 / 8.0)
    t /= t.sum()
    np.testing.assert_allclose(g, np.outer(t, t), rtol=1e-14)


def test_filter_valid_matches_scipy(orc):
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(19, 23))
    g = rng.uniform(size=(5, 5))
    out = orc.filter_valid(img, g, 2)
    np.testing.assert_allclose(out, correlate2d(img, g, mode="valid"), rtol=1e-13)


def test_filter_of_constant_is_constant(orc):
    g = orc.gauss_window(2.0, 5)
    out = orc.filter_valid(np.full((20, 20), 0.3), g, 5)
    np.testing.assert_allclose(out, 0.3, rtol=1e-14)


def test_mse_zero_when_equal(orc):
    h = (np.random.default_rng(1).uniform(size=(2, 16, 16)) > 0.5).astype(np.float64)
    r = orc.reward(h, h)
    assert np.all(r[:, 0] == 0.0)


def test_mse_matches_scipy_filtering(orc):
    rng = np.random.default_rng(2)
    c = synth.contone(9, 24, 30).astype(np.float64)
    h = (rng.uniform(size=c.shape) < c).astype(np.float64)
    G = orc.gauss_window(2.0, 5)
    e = correlate2d(h, G, mode="valid") - correlate2d(c, G, mode="valid")
    r = orc.reward(h, c)
    assert abs(r[0, 0] - np.mean(e * e)) < 1e-15


def test_mse_of_checkerboard_on_half_gray(orc):
    # h = checkerboard, c = 0.5: F(h) - 0.5 = +-(1/2)(sum_i (-1)^i g_i)^2 at
    # every valid pixel (separable window), so MSE = (1/4) s^4 with s the
    # alternating sum of the normalised 1-D profile
    H = W = 20
    yy, xx = np.mgrid[0:H, 0:W]
    h = ((yy + xx) % 2).astype(np.float64)
    c = np.full((H, W), 0.5)
    t = np.exp(-np.arange(-5, 6) ** 2 / 8.0)
    t /= t.sum()
    s = np.sum(t * (-1.0) ** np.arange(11))
    r = orc.reward(h, c)
    assert abs(r[0, 0] - 0.25 * s ** 4) < 1e-15


def test_ssim_of_identical_images_is_one(orc):
    # h = c, real-valued: SSIM = 1 everywhere, so CSSIM = 1
    c = synth.contone(4, 26, 26).astype(np.float64)
    r = orc.reward(c, c)
    assert abs(r[0, 1] - 1.0) < 1e-14


def test_cssim_is_one_on_flat_contone(orc):
    # sigma_c = 0 where the contone window is constant: CSSIM = 1 for any h
    rng = np.random.default_rng(3)
    c = np.full((1, 21, 21), 0.37)
    h = (rng.uniform(size=c.shape) > 0.4).astype(np.float64)
    r = orc.reward(h, c)
    assert abs(r[0, 1] - 1.0) < 1e-15
    assert abs(r[0, 2] - (-r[0, 0] + 0.06)) < 1e-15


def test_constant_images(orc):
    # h = a and c = b constant: HVS-MSE = (a - b)^2, and sigma_c = 0 makes
    # CSSIM = 1 whatever SSIM is
    a, b = 0.2, 0.7
    h = np.full((1, 11, 11), a)
    c = np.full((1, 11, 11), b)
    r = orc.reward(h, c, dict(w_s=1.0))
    assert abs(r[0, 1] - 1.0) < 1e-15
    assert abs(r[0, 0] - (a - b) ** 2) < 1e-15


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.1), (0.5, 0.2), (2.0, -0.3)])
def test_ssim_affine_closed_form(orc, alpha, beta):
    # 3x3 image, radius-1 window, single valid pixel (the centre).
    # With h = alpha*c + beta: mu_h = alpha mu_c + beta, var_h = alpha^2 var_c,
    # cov = alpha var_c. Hence
    # SSIM = (2 mu_h mu_c + C1)(2 alpha var_c + C2) /
    #        ((mu_h^2 + mu_c^2 + C1)((1 + alpha^2) var_c + C2)),
    # CSSIM = sigma SSIM + 1 - sigma with sigma = 2 sqrt(var_c).
    rng = np.random.default_rng(4)
    c = rng.uniform(0.2, 0.8, size=(3, 3))
    h = alpha * c + beta
    prm = dict(hvs_r=1, ssim_r=1, ssim_sigma=1.5, w_s=1.0)
    w = orc.gauss_window(1.5, 1)
    mu_c = np.sum(w * c)
    var_c = np.sum(w * (c - mu_c) ** 2)
    mu_h = alpha * mu_c + beta
    C1, C2 = 1e-4, 9e-4
    ssim = (2 * mu_h * mu_c + C1) * (2 * alpha * var_c + C2) / (
        (mu_h ** 2 + mu_c ** 2 + C1) * ((1 + alpha ** 2) * var_c + C2))
    sig = 2.0 * math.sqrt(var_c)
    r = orc.reward(h[None], c[None], prm)
    assert abs(r[0, 1] - (sig * ssim + 1 - sig)) < 1e-14


def test_contrast_map_in_unit_interval(orc):
    # sigma_c = 2 sqrt(var) <= 1 for c in [0,1]; the extreme half black/half
    # white window reaches close to 1. CSSIM of h = 1 - c is then < 1.
    H = W = 11
    c = np.zeros((1, H, W))
    c[0, :, 6:] = 1.0
    c[0, :, 5] = 0.5
    w = orc.gauss_window(1.5, 5)
    mu = np.sum(w * c[0])
    var = np.sum(w * (c[0] - mu) ** 2)
    assert 0.0 <= 2 * math.sqrt(var) <= 1.0
    r = orc.reward(1.0 - c, c, dict(w_s=1.0))
    assert r[0, 1] < 1.0


def test_reward_combination(orc):
    rng = np.random.default_rng(5)
    c = synth.contone(11, 18, 18).astype(np.float64)
    h = (rng.uniform(size=c.shape) < c).astype(np.float64)
    r = orc.reward(h, c, dict(w_s=0.06))
    assert abs(r[0, 2] - (-r[0, 0] + 0.06 * r[0, 1])) < 1e-16
