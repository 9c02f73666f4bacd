"""GPU parity of halftone_spectrum (mean-periodogram RAPSD and anisotropy,
Sec. IV) against the oracle: RAPSD to 1e-5 relative, anisotropy to 1e-4
relative plus 1e-6 absolute (an FP32 DFT of 0/1 patches against FP64)."""
import numpy as np
import pytest
import torch

from gpu_common import to_dev
from paper_2304_12152_amd import binding as hb

pytestmark = pytest.mark.gpu


def _bits(seed, B, H, W, gray):
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=(B, H, W)) < gray).astype(np.uint8)


def _check(orc, bits, P):
    r, a = hb.halftone_spectrum(to_dev(bits), P)
    torch.cuda.synchronize()
    rr, ra = orc.spectrum(bits.astype(np.float64), P)
    np.testing.assert_allclose(r.cpu().numpy(), rr, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(a.cpu().numpy(), ra, rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("P", [32, 64])
@pytest.mark.parametrize("shape,gray", [((1, 64, 64), 0.5), ((3, 100, 130), 0.06),
                                        ((2, 130, 200), 0.39)])
def test_spectrum_matches_oracle_on_white_noise(orc, P, shape, gray):
    _check(orc, _bits(P + shape[1], *shape, gray), P)


@pytest.mark.parametrize("P", [32, 64])
def test_spectrum_of_error_diffusion(orc, P):
    # structured halftones: Floyd-Steinberg at the evaluation gray levels
    grays = np.array([15, 80, 100, 127], dtype=np.float64) / 255.0
    n = 128 if P == 32 else 64
    c = np.broadcast_to(grays[:, None, None], (4, n, 128)).copy()
    bits = orc.floyd_steinberg(c).astype(np.uint8)
    _check(orc, bits, P)


def test_spectrum_single_patch_and_degenerate_inputs(orc):
    # exactly one patch; an all-zero batch (every ring has zero power: A = 0);
    # an all-one batch (only the DC ring carries power, up to the rounding
    # of the FP32 twiddles elsewhere)
    _check(orc, _bits(5, 1, 32, 32, 0.3), 32)
    z = np.zeros((2, 64, 64), dtype=np.uint8)
    r, a = hb.halftone_spectrum(to_dev(z), 32)
    assert not r.any() and not a.any()
    o = np.ones((1, 64, 96), dtype=np.uint8)
    r, a = hb.halftone_spectrum(to_dev(o), 32)
    r = r.cpu().numpy()
    assert r[0] == pytest.approx(32.0 * 32.0, rel=1e-6) and np.abs(r[1:]).max() < 1e-6


def test_spectrum_at_full_page_size(orc):
    # a 1024 x 1040 page tiled 4 x 4 by one 256 x 256 block (ragged 16-column
    # tail dropped): every patch of the page repeats one of the block's 64
    # patches 16 times, so the page's mean periodogram is the block's
    blk = _bits(11, 1, 256, 256, 0.25)
    page = np.zeros((1, 1024, 1040), dtype=np.uint8)
    page[:, :, :1024] = np.tile(blk, (1, 4, 4))
    page[:, :, 1024:] = 1
    r, a = hb.halftone_spectrum(to_dev(page), 32)
    rr, ra = orc.spectrum(blk.astype(np.float64), 32)
    np.testing.assert_allclose(r.cpu().numpy(), rr, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(a.cpu().numpy(), ra, rtol=1e-4, atol=1e-6)
