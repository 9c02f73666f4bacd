"""Pins of the oracle's random draws: Philox4x32-10 against its published
known-answer vectors, and the statistics of the uniform, Gaussian and
Bernoulli draws built on it."""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(orc, row):
    ctr, key, want = row
    got = orc.philox(ctr, key)
    assert [int(x) for x in got] == want


def test_uniform_chi_square(orc):
    # 10^6 draws into 100 equal bins; chi^2 with 99 dof has mean 99, sd 14.
    z = orc.noise_map([12345], 1000, 1000, kind=1, stream=4, step=0).ravel()
    assert z.min() >= 0.0 and z.max() < 1.0
    counts = np.histogram(z, bins=100, range=(0.0, 1.0))[0]
    chi2 = ((counts - 1e4) ** 2 / 1e4).sum()
    assert chi2 < 99 + 6 * 14
    # every draw is a multiple of 2^-24 (exactly representable in FP32)
    assert np.all(z * 2.0 ** 24 == np.floor(z * 2.0 ** 24))


def test_normal_moments_and_tails(orc):
    z = orc.noise_map([7, 8], 500, 1000, kind=0, stream=1, step=3).ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    # fraction beyond 2 sigma: 0.0455 for N(0,1)
    frac = np.mean(np.abs(z) > 2.0)
    assert abs(frac - 0.0455) < 5.0 * math.sqrt(0.0455 * 0.9545 / n)
    # symmetric third moment
    assert abs(np.mean(z ** 3)) < 5.0 * math.sqrt(15.0 / n)


def test_streams_and_steps_are_independent(orc):
    a = orc.noise_map([5], 64, 64, kind=1, stream=1, step=0).ravel()
    b = orc.noise_map([5], 64, 64, kind=1, stream=0, step=0).ravel()
    c = orc.noise_map([5], 64, 64, kind=1, stream=1, step=1).ravel()
    d = orc.noise_map([6], 64, 64, kind=1, stream=1, step=0).ravel()
    for other in (b, c, d):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.06


@pytest.mark.parametrize("g", [15 / 255, 0.25, 0.5, 0.8])
def test_bernoulli_fill_fraction(orc, g):
    # constant probability g: the expected fill of white is g (tone
    # preservation); binomial bound 4 sd
    N = 256 * 256
    p = np.full((1, 256, 256), g)
    h = orc.bernoulli(p, [99], step=2)
    assert abs(h.mean() - g) <= 4.0 * math.sqrt(g * (1 - g) / N)


def test_bernoulli_is_u_below_p(orc):
    p = np.random.default_rng(0).uniform(size=(2, 16, 16))
    h = orc.bernoulli(p, [3, 4], step=9)
    u = np.stack([orc.noise_map([s], 16, 16, kind=1, stream=0, step=9)[0] for s in (3, 4)])
    assert np.array_equal(h, (u < p).astype(np.uint8))
