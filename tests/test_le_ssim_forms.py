"""The two FP32 forms of a toggle's SSIM change in the Local Expectation
gradient (Sec. III-C): the cancellation-free difference of le_grad_kernel
and the direct A'B'/(C'D') - SSIM_j of the register-blocked binary kernel.
Both are checked in FP64 against the plain definition (the SSIM maps of
the toggled halftone recomputed by brute force), and in FP32 against the
FP64 value: the direct form's error must stay within a small factor of the
cancellation-free form's, both being set by the rounding of the FP32 window
statistics. CPU only, numpy emulation of the kernels' arithmetic."""
import numpy as np
from scipy.signal import correlate2d

from paper_2304_12152_amd import synth

C1, C2, K = 1e-4, 9e-4, 2.0
R = 5


def _window(sigma=1.5, r=R):
    i = np.arange(-r, r + 1)
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2 * sigma * sigma))
    return g / g.sum()


def _stats(h, c, w):
    f = lambda x: correlate2d(x, w, mode="same", boundary="fill")
    mh, mc = f(h), f(c)
    vc = np.maximum(f(c * c) - mc * mc, 0.0)
    cov = f(h * c) - mh * mc
    return mh, mc, vc, cov


def _ssim(mh, mc, vc, cov):
    vh = mh * (1 - mh)
    return ((2 * mh * mc + C1) * (2 * cov + C2)) / ((mh * mh + mc * mc + C1) * (vh + vc + C2))


def _case(H=48, W=52, seed=7):
    c = synth.contone(seed, H, W).astype(np.float64)
    rng = np.random.default_rng(seed)
    h = (c + 0.3 * rng.standard_normal(c.shape) > 0.5).astype(np.float64)
    return h, c, _window()


def _toggle_sums(h, c, w, dt, direct):
    """Sum over the 121 centres j of sigma_j (SSIM_j(h with a toggled) -
    SSIM_j(h)) for every pixel a at least 2R from the border, in type dt."""
    H, W = h.shape
    mh, mc, vc, cov = (x.astype(dt) for x in _stats(h, c, w))
    one, two = dt(1), dt(2)
    sg = dt(K) * np.sqrt(vc)
    A = two * mh * mc + dt(C1)
    B = two * cov + dt(C2)
    C = mh * mh + mc * mc + dt(C1)
    D = mh * (one - mh) + vc + dt(C2)
    S = (A * B) * (one / (C * D))
    ys, xs = np.mgrid[2 * R:H - 2 * R, 2 * R:W - 2 * R]
    delta = np.where(h[ys, xs] != 0, dt(-1), one)
    ca = c[ys, xs].astype(dt)
    acc = np.zeros(ys.shape, dt)
    for i in range(-R, R + 1):
        for j in range(-R, R + 1):
            jy, jx = ys + i, xs + j
            dw = delta * dt(w[R - i, R - j])
            a, b, cc, d = A[jy, jx], B[jy, jx], C[jy, jx], D[jy, jx]
            m_h, m_c = mh[jy, jx], mc[jy, jx]
            dA, dB = two * dw * m_c, two * dw * (ca - m_c)
            dC, dD = dw * (two * m_h + dw), dw * (one - two * m_h - dw)
            if direct:
                t = ((a + dA) * (b + dB)) * (one / ((cc + dC) * (d + dD))) - S[jy, jx]
            else:
                num = cc * d * (a * dB + b * dA + dA * dB) - a * b * (cc * dD + d * dC + dC * dD)
                t = num * (one / ((cc + dC) * (d + dD) * (cc * d)))
            acc = acc + sg[jy, jx] * t
    return acc, (ys, xs)


def test_both_forms_are_the_toggled_ssim_change_in_fp64():
    h, c, w = _case(H=36, W=36)
    ref_free, (ys, xs) = _toggle_sums(h, c, w, np.float64, direct=False)
    ref_direct, _ = _toggle_sums(h, c, w, np.float64, direct=True)
    scale = np.abs(ref_free).max()
    assert np.abs(ref_direct - ref_free).max() < 1e-12 * scale
    # brute force: the SSIM maps of the toggled halftone, for a few pixels
    mh, mc, vc, cov = _stats(h, c, w)
    s0 = _ssim(mh, mc, vc, cov)
    sg = K * np.sqrt(vc)
    for (py, px) in [(0, 0), (3, 7), (8, 2), (ys.shape[0] - 1, ys.shape[1] - 1)]:
        ay, ax = ys[py, px], xs[py, px]
        ht = h.copy()
        ht[ay, ax] = 1 - ht[ay, ax]
        # sigma_j is the contone's, so it does not change with the toggle
        d = (sg * (_ssim(*_stats(ht, c, w)) - s0))[ay - R:ay + R + 1, ax - R:ax + R + 1].sum()
        assert abs(d - ref_free[py, px]) < 1e-12 * scale


def test_direct_form_fp32_error_matches_the_cancellation_free_form():
    h, c, w = _case()
    ref, _ = _toggle_sums(h, c, w, np.float64, direct=False)
    scale = np.abs(ref).max()
    e_free = np.abs(_toggle_sums(h, c, w, np.float32, direct=False)[0] - ref).max() / scale
    e_direct = np.abs(_toggle_sums(h, c, w, np.float32, direct=True)[0] - ref).max() / scale
    assert e_free < 2e-6 and e_direct < 2e-6
    assert e_direct < 3.0 * e_free
