"""Pins of the anisotropy-suppressing loss (Sec. IV, Eqs. psd, rapsd, as):
ring geometry, closed forms (constant patch, Parseval, a single cosine),
transpose invariance, numpy's FFT, and finite differences of the adjoint."""
import numpy as np
import pytest

RING_COUNTS_32 = [1, 8, 12, 16, 32, 28, 40, 40, 48, 68, 56, 72, 68, 88, 88, 84, 94, 64, 44,
                  32, 16, 20, 4, 1]


def test_ring_counts(orc):
    counts = np.zeros(24, dtype=int)
    for u in range(32):
        for v in range(32):
            counts[orc.ring_index(u, v, 32)] += 1
    assert counts.tolist() == RING_COUNTS_32
    assert counts.sum() == 1024


def test_ring_is_rounded_radius(orc):
    for u in range(32):
        for v in range(32):
            ub, vb = min(u, 32 - u), min(v, 32 - v)
            assert orc.ring_index(u, v, 32) == int(np.floor(np.hypot(ub, vb) + 0.5))


def test_constant_patch_has_zero_loss_and_gradient(orc):
    x = np.full((2, 64, 64), 0.37)
    L, g = orc.as_loss(x)
    assert abs(L) < 1e-18 * 1024 ** 2
    assert np.abs(g).max() < 1e-12


def _periodogram(patch):
    X = np.fft.fft2(patch)
    return np.abs(X) ** 2 / patch.size


def _loss_numpy(xmap, P=32):
    B, H, W = xmap.shape
    rho = np.array([[int(np.floor(np.hypot(min(u, P - u), min(v, P - v)) + 0.5))
                     for v in range(P)] for u in range(P)])
    tot, n = 0.0, 0
    for b in range(B):
        for ty in range(H // P):
            for tx in range(W // P):
                ph = _periodogram(xmap[b, ty * P:(ty + 1) * P, tx * P:(tx + 1) * P])
                for r in range(rho.max() + 1):
                    m = rho == r
                    tot += np.sum((ph[m] - ph[m].mean()) ** 2)
                n += 1
    return tot / n


def test_single_cosine_closed_form(orc):
    # x = cos(2 pi 4 x / 32): X(0,4) = X(0,28) = 512, Phat = 256 at those two
    # bins of ring 4 (32 samples), ring mean 16, so
    # L = 2 (256 - 16)^2 + 30 * 16^2 = 122880.
    xx = np.arange(32)
    x = np.broadcast_to(np.cos(2 * np.pi * 4 * xx / 32)[None, :], (32, 32)).copy()
    L, _ = orc.as_loss(x[None])
    assert abs(L - 122880.0) < 1e-6


def test_matches_numpy_fft(orc):
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(2, 64, 96))
    L, _ = orc.as_loss(x)
    assert abs(L - _loss_numpy(x)) < 1e-9 * abs(L)


def test_parseval_and_transpose_invariance(orc):
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(32, 32))
    assert abs(_periodogram(x).sum() - np.sum(x * x)) < 1e-10
    L1, _ = orc.as_loss(x[None])
    L2, _ = orc.as_loss(x.T.copy()[None])
    assert abs(L1 - L2) < 1e-9 * L1


def test_remainders_are_dropped(orc):
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(1, 45, 70))
    L, g = orc.as_loss(x)
    L2, _ = orc.as_loss(x[:, :32, :64].copy())
    assert abs(L - L2) < 1e-10 * L
    assert np.all(g[:, 32:, :] == 0.0) and np.all(g[:, :, 64:] == 0.0)


def test_adjoint_finite_differences(orc):
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(2, 32, 64))
    L, g = orc.as_loss(x)
    eps = 1e-5
    for _ in range(12):
        b, y, xx = rng.integers(2), rng.integers(32), rng.integers(64)
        xp = x.copy(); xp[b, y, xx] += eps
        xm = x.copy(); xm[b, y, xx] -= eps
        fd = (orc.as_loss(xp, grad=False)[0] - orc.as_loss(xm, grad=False)[0]) / (2 * eps)
        assert abs(fd - g[b, y, xx]) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_adjoint_is_two_re_ifft(orc):
    # dL_patch/dx = 2 Re(ifft2(g * X)), g = 2 (Phat - Pbar), one patch
    rng = np.random.default_rng(4)
    x = rng.uniform(size=(32, 32))
    L, grad = orc.as_loss(x[None])
    X = np.fft.fft2(x)
    ph = np.abs(X) ** 2 / 1024
    rho = np.array([[orc.ring_index(u, v, 32) for v in range(32)] for u in range(32)])
    pbar = np.zeros_like(ph)
    for r in range(24):
        pbar[rho == r] = ph[rho == r].mean()
    want = 2 * np.real(np.fft.ifft2(2 * (ph - pbar) * X))
    np.testing.assert_allclose(grad[0], want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_anisotropy_of_white_noise_is_near_zero_db(orc):
    # for a white-noise periodogram each bin is ~ exponential, so the ring
    # variance over squared mean is ~1 (0 dB); averaged over many patches.
    rng = np.random.default_rng(5)
    acc = np.zeros(24)
    n = 40
    for _ in range(n):
        p = (rng.uniform(size=(32, 32)) < 0.5).astype(np.float64) - 0.5
        _, a = orc.anisotropy(p)
        acc += a
    mean_mid = (acc / n)[4:16].mean()
    assert 0.7 < mean_mid < 1.3
