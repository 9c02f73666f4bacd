"""Pins of the oracle's multitoning prototype (Sec. VI-E, its unnumbered rounding equation):
L = 2 is the binary method, the local toggle equals brute force, the
actions are the unbiased stochastic rounding between adjacent levels, the
test phase rounds to the nearest level, and the estimator is the exact
derivative of the expected reward (enumeration of every action)."""
import itertools

import numpy as np
import pytest

SMALL = dict(hvs_r=1, ssim_r=1)


def _v(rng, shape):
    # values away from the level boundaries of L = 2, 3, 4
    v = rng.uniform(0.02, 0.98, size=shape)
    return v


def test_two_levels_are_the_binary_method(orc):
    rng = np.random.default_rng(0)
    v = _v(rng, (2, 13, 15))
    seeds = [5, 9]
    np.testing.assert_array_equal(orc.multitone_actions(v, seeds, 2, step=3),
                                  orc.bernoulli(v, seeds, step=3))
    x = rng.normal(0, 3, size=(2, 13, 15))
    x[0, 0, :3] = [0.0, -1e-300, 1e-300]
    np.testing.assert_array_equal(orc.multitone_levels(x, 2), orc.threshold(x))
    c = rng.uniform(0, 1, size=(2, 13, 15))
    h = orc.bernoulli(v, seeds).astype(np.float64)
    np.testing.assert_allclose(orc.multitone_delta(h, c, v, 2), orc.le_delta(h, c),
                               rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("L", [3, 4, 8])
@pytest.mark.parametrize("prm,shape", [(SMALL, (1, 6, 7)), (None, (2, 14, 15))])
def test_local_toggle_equals_brute_force(orc, L, prm, shape):
    rng = np.random.default_rng(L)
    v = rng.uniform(0, 1, size=shape)
    c = rng.uniform(0, 1, size=shape)
    k = orc.multitone_actions(v, list(range(shape[0])), L)
    h = k / (L - 1.0)
    loc = orc.multitone_delta(h, c, v, L, prm)
    bru = orc.multitone_delta(h, c, v, L, prm, brute=True)
    np.testing.assert_allclose(loc, bru, rtol=1e-10, atol=1e-14 * np.abs(bru).max())
    assert np.abs(bru).max() > 0


@pytest.mark.parametrize("L", [3, 4])
def test_actions_are_unbiased_rounding_between_adjacent_levels(orc, L):
    rng = np.random.default_rng(1)
    v = rng.uniform(0, 1, size=(1, 200, 200))
    k = orc.multitone_actions(v, [3], L).astype(int)
    kf = np.minimum(np.floor(v * (L - 1)).astype(int), L - 2)
    assert np.all((k == kf) | (k == kf + 1))
    # constant v: the mean level equals v within 4 sigma of the binomial
    for val in (0.4, 0.9, 1.0 / 7.0):
        vv = np.full((1, 300, 300), val)
        kk = orc.multitone_actions(vv, [11], L)
        kf0 = min(int(np.floor(val * (L - 1))), L - 2)
        q = val * (L - 1) - kf0
        sd = np.sqrt(q * (1 - q) / kk.size) / (L - 1)
        assert abs(kk.mean() / (L - 1) - val) <= 4 * sd + 1e-12
    # the ends and the levels themselves are drawn with probability one
    for val, want in ((0.0, 0), (1.0, L - 1), (1.0 / (L - 1), 1)):
        kk = orc.multitone_actions(np.full((1, 50, 50), val), [2], L)
        assert np.all(kk == want)


def test_levels_round_to_the_nearest_with_ties_up(orc):
    L = 4
    logit = lambda p: np.log(p / (1.0 - p))
    v = np.array([1e-9, 1 / 6 - 1e-6, 1 / 6 + 1e-6, 1 / 3, 0.5 - 1e-6, 0.5, 5 / 6 + 1e-6,
                  1 - 1e-9])
    got = orc.multitone_levels(logit(v), L)
    np.testing.assert_array_equal(got, [0, 0, 1, 1, 1, 2, 3, 3])


@pytest.mark.parametrize("L", [3, 4])
def test_estimator_is_the_derivative_of_the_expected_reward(orc, L):
    # 3 x 3 image, 3 x 3 windows: the one valid reward pixel sees every agent
    rng = np.random.default_rng(7 + L)
    prm = dict(SMALL, w_s=0.5)
    v = rng.uniform(0.05, 0.95, size=(1, 3, 3))
    # keep every v inside its rounding cell by 1e-3 for the difference quotient
    cell = v * (L - 1) - np.floor(v * (L - 1))
    v = np.where(cell < 0.01, v + 0.02 / (L - 1), v)
    v = np.where(cell > 0.99, v - 0.02 / (L - 1), v)
    c = rng.uniform(0, 1, size=(1, 3, 3))
    kf = np.floor(v * (L - 1)).astype(int).ravel()
    q = (v * (L - 1)).ravel() - kf

    def expected(qv, with_grad):
        er, g = 0.0, np.zeros(9)
        for bits in itertools.product((0, 1), repeat=9):
            b = np.array(bits)
            pr = np.prod(np.where(b == 1, qv, 1 - qv))
            h = ((kf + b) / (L - 1.0)).reshape(1, 3, 3)
            er += pr * orc.reward(h, c, prm)[0, 2]
            if with_grad:
                g += pr * orc.multitone_delta(h, c, v, L, prm).ravel() * (L - 1)
        return er, g

    _, g = expected(q, True)
    eps = 1e-4
    fd = np.zeros(9)
    for a in range(9):
        qp, qm = q.copy(), q.copy()
        qp[a] += eps * (L - 1)
        qm[a] -= eps * (L - 1)
        fd[a] = (expected(qp, False)[0] - expected(qm, False)[0]) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-12)
