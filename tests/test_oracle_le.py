"""Pins of the Local Expectation gradient (Sec. III-B/C): the efficient local
toggle form against brute-force re-evaluation of R, and the estimator's
unbiasedness by exhaustive enumeration of every halftone of a 4x4 image."""
import itertools

import numpy as np
import pytest

from paper_2304_12152_amd import synth


@pytest.mark.parametrize("prm", [dict(), dict(w_s=1.0), dict(hvs_r=2, ssim_r=3, w_s=0.5),
                                 dict(hvs_r=3, ssim_r=1, w_s=2.0)])
def test_local_equals_brute_force(orc, prm):
    rng = np.random.default_rng(0)
    c = synth.contone_batch([21, 22], 16, 18).astype(np.float64)
    h = (rng.uniform(size=c.shape) < c).astype(np.float64)
    brute = orc.le_delta(h, c, prm, brute=True)
    local = orc.le_delta(h, c, prm, brute=False)
    scale = np.abs(brute).max()
    assert scale > 0
    np.testing.assert_allclose(local, brute, rtol=0, atol=1e-12 * max(scale, 1e-3))


def test_local_equals_brute_force_on_flats(orc):
    # saturated flats (c = 0 or 1 in most of the window): sigma_c = 0 there
    c = np.zeros((1, 14, 14))
    c[0, :, 7:] = 1.0
    h = np.zeros_like(c)
    h[0, ::3, ::2] = 1.0
    brute = orc.le_delta(h, c, dict(w_s=1.0), brute=True)
    local = orc.le_delta(h, c, dict(w_s=1.0), brute=False)
    np.testing.assert_allclose(local, brute, rtol=0, atol=1e-13)


def test_delta_mse_toggle_is_exact_quadratic(orc):
    # with w_s = 0, R = -MSE; the toggle of pixel a changes the MSE by exactly
    # (1/M) sum_j (2 delta G e_j + G^2): check by recomputing R after the flip
    rng = np.random.default_rng(1)
    c = rng.uniform(size=(1, 15, 15))
    h = (rng.uniform(size=c.shape) < 0.5).astype(np.float64)
    prm = dict(w_s=0.0)
    d = orc.le_delta(h, c, prm)
    r0 = orc.reward(h, c, prm)[0, 2]
    for (y, x) in [(7, 7), (0, 0), (3, 12), (14, 5)]:
        t = h.copy()
        t[0, y, x] = 1.0 - t[0, y, x]
        r1 = orc.reward(t, c, prm)[0, 2]
        delta = 1.0 - 2.0 * h[0, y, x]
        assert abs(delta * (r1 - r0) - d[0, y, x]) < 1e-15


def test_le_estimator_is_unbiased_by_enumeration(orc):
    # 4x4 image, radius-1 windows (valid region 2x2). For every pixel a,
    # E_{h~pi}[dR_a(h)] must equal dE_pi[R]/dp_a (Eq. halftoners). E_pi[R] is
    # multilinear in p, so its central difference is exact up to rounding.
    prm = dict(hvs_r=1, ssim_r=1, hvs_sigma=1.0, ssim_sigma=1.0, w_s=1.0)
    rng = np.random.default_rng(2)
    c = rng.uniform(0.1, 0.9, size=(4, 4))
    p = rng.uniform(0.1, 0.9, size=16)
    H = np.array(list(itertools.product([0.0, 1.0], repeat=16)))  # 65536 x 16
    hs = H.reshape(-1, 4, 4)
    cs = np.broadcast_to(c, hs.shape).copy()
    R = orc.reward(hs, cs, prm)[:, 2]
    dR = orc.le_delta(hs, cs, prm).reshape(-1, 16)

    def prob(pv):
        return np.prod(np.where(H == 1.0, pv, 1.0 - pv), axis=1)

    pi = prob(p)
    lhs = pi @ dR
    eps = 1e-3
    for a in range(16):
        pp = p.copy(); pp[a] += eps
        pm = p.copy(); pm[a] -= eps
        rhs = (prob(pp) @ R - prob(pm) @ R) / (2 * eps)
        assert abs(lhs[a] - rhs) < 1e-12 * max(1.0, abs(rhs)) + 1e-13


def test_grad_probs_is_minus_delta_over_batch(orc):
    rng = np.random.default_rng(3)
    c = rng.uniform(size=(3, 12, 12))
    h = (rng.uniform(size=c.shape) < c).astype(np.float64)
    d = orc.le_delta(h, c)
    g = orc.le_grad_probs(h, c)
    np.testing.assert_array_equal(g, -d / 3)


def test_policy_gradient_prefers_the_two_dithers_of_half_gray(orc):
    # The toy of Fig. 1: a contone of constant 0.5 is best reproduced by
    # alternating dots. With per-pixel logits trained by the Local
    # Expectation gradient on a flat 0.5 image, R rises from the p = 0.5
    # start and the expected fill stays at 0.5.
    prm = dict(w_s=0.0, hvs_r=1, ssim_r=1, hvs_sigma=1.0, ssim_sigma=1.0)
    Hh = Ww = 8
    c = np.full((1, Hh, Ww), 0.5)
    theta = np.zeros((1, Hh, Ww))
    rng = np.random.default_rng(4)

    def expected_reward(th, n=64):
        p = 1.0 / (1.0 + np.exp(-th))
        h = (rng.uniform(size=(n, Hh, Ww)) < p).astype(np.float64)
        return orc.reward(h, np.broadcast_to(c, h.shape).copy(), prm)[:, 2].mean()

    r_start = expected_reward(theta)
    for it in range(300):
        p = 1.0 / (1.0 + np.exp(-theta))
        h = (rng.uniform(size=p.shape) < p).astype(np.float64)
        g = -orc.le_delta(h, c, prm)  # dL/dp for B = 1
        theta -= 2000.0 * g * p * (1 - p)
    r_end = expected_reward(theta)
    p = 1.0 / (1.0 + np.exp(-theta))
    assert r_end > r_start
    assert abs(p.mean() - 0.5) < 0.1
    # bimodal: the policy has committed to a binary pattern
    assert np.mean((p < 0.1) | (p > 0.9)) > 0.8
