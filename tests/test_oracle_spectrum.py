"""Pins of the blue-noise spectral measures (Sec. IV, Eqs. psd, rapsd,
anis) as the evaluation uses them: the power spectrum estimated by the mean
of the periodograms of non-overlapping patches."""
import numpy as np


def test_single_patch_equals_the_per_patch_measure(orc):
    rng = np.random.default_rng(7)
    p = (rng.uniform(size=(32, 32)) < 0.3).astype(np.float64)
    r1, a1 = orc.spectrum(p, 32)
    r2, a2 = orc.anisotropy(p)
    np.testing.assert_allclose(r1, r2, rtol=1e-12)
    np.testing.assert_allclose(a1, a2, rtol=1e-12, atol=1e-15)


def test_repeated_patches_average_to_the_same_spectrum(orc):
    rng = np.random.default_rng(8)
    p = (rng.uniform(size=(32, 32)) < 0.6).astype(np.float64)
    tiled = np.tile(p, (2, 3))  # 64 x 96: six copies of the patch
    r1, a1 = orc.spectrum(tiled, 32)
    r2, a2 = orc.spectrum(p, 32)
    np.testing.assert_allclose(r1, r2, rtol=1e-12)
    np.testing.assert_allclose(a1, a2, rtol=1e-12, atol=1e-15)


def test_parseval_on_the_mean_periodogram(orc):
    # sum over f of P(f) = sum over the patch of x^2 (Parseval, with the 1/N of
    # Eq. psd), so ring sums of the RAPSD times ring sizes add up to the mean
    # over patches of sum x^2
    rng = np.random.default_rng(9)
    img = (rng.uniform(size=(2, 64, 64)) < 0.4).astype(np.float64)
    r, _ = orc.spectrum(img, 32)
    counts = np.zeros(len(r))
    for u in range(32):
        for v in range(32):
            counts[orc.ring_index(u, v, 32)] += 1
    total = (r * counts).sum()
    patches = img.reshape(2, 2, 32, 2, 32).transpose(0, 1, 3, 2, 4).reshape(-1, 32, 32)
    assert abs(total - (patches ** 2).sum(axis=(1, 2)).mean()) < 1e-9


def test_checkerboard_closed_form(orc):
    # x = (1 + (-1)^(x + y)) / 2: X(0, 0) = N / 2 and X(P/2, P/2) = N / 2, so
    # P = N / 4 at both; every other bin is 0. The Nyquist bin is alone in
    # its ring only if no other (u, v) rounds to the same radius.
    P = 32
    y, x = np.mgrid[0:P, 0:P]
    cb = ((x + y) % 2 == 0).astype(np.float64)
    r, a = orc.spectrum(cb, P)
    ring = orc.ring_index(P // 2, P // 2, P)
    n = sum(orc.ring_index(u, v, P) == ring for u in range(P) for v in range(P))
    assert abs(r[0] - P * P / 4) < 1e-9
    assert abs(r[ring] - (P * P / 4) / n) < 1e-9
    others = [k for k in range(len(r)) if k not in (0, ring)]
    assert np.abs(r[others]).max() < 1e-9


def test_white_noise_anisotropy_falls_as_one_over_k(orc):
    # each bin of a white-noise periodogram is exponential (variance = mean^2),
    # so the mean of K periodograms has anisotropy about 1 / K, and the RAPSD
    # is the variance 1/4 of a fair coin (ring 0 holds the mean's power)
    rng = np.random.default_rng(10)
    K = 16
    img = (rng.uniform(size=(K, 32, 32)) < 0.5).astype(np.float64)
    r, a = orc.spectrum(img, 32)
    mid = a[4:16]
    assert 0.6 / K < mid.mean() < 1.5 / K
    assert abs(r[4:16].mean() - 0.25) < 0.03
