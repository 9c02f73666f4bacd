"""GPU parity of halftone_loss / halftone_loss_backward against the oracle:
reward terms and L_AS to 1e-5 relative, Local Expectation and anisotropy
gradients to 1e-4 of their largest entry."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import device, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import synth

pytestmark = pytest.mark.gpu


def _case(seeds, H, W, pseed=0):
    c = synth.contone_batch(seeds, H, W)
    rng = np.random.default_rng(pseed)
    # probabilities with a realistic spread around the contone
    p = np.clip(c + rng.normal(0, 0.2, size=c.shape), 0.01, 0.99).astype(np.float32)
    h = (rng.uniform(size=c.shape) < p).astype(np.uint8)
    return c, p, h


@pytest.mark.parametrize("shape", [(1, 11, 11), (3, 40, 52), (2, 256, 256), (1, 23, 300)])
def test_loss_matches_oracle(orc, shape):
    B, H, W = shape
    c, p, h = _case(range(100, 100 + B), H, W)
    out = hb.halftone_loss(to_dev(h), to_dev(c)).cpu().numpy()
    ref = orc.reward(h.astype(np.float64), c.astype(np.float64))
    np.testing.assert_allclose(out[:3 * B].reshape(B, 3), ref, rtol=1e-5, atol=1e-8)
    assert out[3 * B] == 0.0
    # the library's total loss, -mean R (no gray batch)
    total = -ref[:, 2].mean()
    assert abs(out[3 * B + 1] - total) <= 1e-5 * abs(total) + 1e-8


def test_loss_with_gray_batch(orc):
    B, H, W = 2, 64, 70
    c, p, h = _case([7, 8], H, W)
    pg = np.clip(np.random.default_rng(3).normal(0.4, 0.3, size=(3, 64, 96)), 0, 1)
    pg = pg.astype(np.float32)
    out = hb.halftone_loss(to_dev(h), to_dev(c), to_dev(pg)).cpu().numpy()
    L, _ = orc.as_loss(pg.astype(np.float64), grad=False)
    assert abs(out[3 * B] - L) <= 1e-5 * abs(L)
    # total loss of the batch: -mean_b R_b + w_a L_AS (Sec. III-B with Sec. IV)
    ref = orc.reward(h.astype(np.float64), c.astype(np.float64))
    total = -ref[:, 2].mean() + 0.002 * L
    assert abs(out[3 * B + 1] - total) <= 1e-5 * abs(total)
    big = hb.default_loss_params(w_a=0.5)
    out2 = hb.halftone_loss(to_dev(h), to_dev(c), to_dev(pg), prm=big).cpu().numpy()
    total2 = -ref[:, 2].mean() + 0.5 * L
    assert abs(out2[3 * B + 1] - total2) <= 1e-5 * abs(total2)


@pytest.mark.parametrize("prm", [dict(), dict(w_s=1.0), dict(hvs_radius=3, ssim_radius=2,
                                                             hvs_sigma=1.2, ssim_sigma=0.9)])
def test_le_gradient_matches_oracle(orc, prm):
    B, H, W = 3, 48, 61
    c, p, h = _case([31, 32, 33], H, W)
    oprm = {("hvs_r" if k == "hvs_radius" else "ssim_r" if k == "ssim_radius" else k): v
            for k, v in prm.items()}
    gp, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c), prm=hb.default_loss_params(**prm))
    gp = gp.cpu().numpy()
    ref = orc.le_grad_probs(h.astype(np.float64), c.astype(np.float64), oprm)
    assert np.abs(gp - ref).max() <= 1e-4 * np.abs(ref).max()
    # logit space multiplies by p (1 - p)
    gl, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c), to_dev(p),
                                      prm=hb.default_loss_params(**prm),
                                      grad_space=hb.HS_WRT_LOGIT)
    refl = ref * p * (1 - p)
    assert np.abs(gl.cpu().numpy() - refl).max() <= 1e-4 * np.abs(refl).max()


@pytest.mark.parametrize("level", [0.0, 0.37, 1.0])
def test_le_gradient_on_flat_contones(orc, level):
    # sigma_c = 0 at every window centre, so the SSIM part of every toggle
    # is weighted by zero and only the HVS part remains (black, a mid gray
    # and white; the binary kernel of the default windows)
    B, H, W = 2, 40, 70
    c = np.full((B, H, W), level, np.float32)
    h = (np.random.default_rng(11).uniform(size=c.shape) < 0.4).astype(np.uint8)
    gp, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c))
    gp = gp.cpu().numpy()
    assert np.isfinite(gp).all()
    ref = orc.le_grad_probs(h.astype(np.float64), c.astype(np.float64))
    assert np.abs(gp - ref).max() <= 1e-4 * np.abs(ref).max()


def test_le_gradient_c3_shape(orc):
    # 16 x 256 x 256 (the loss workload): every image's full map against the
    # oracle's, the whole batch in one oracle call (same -dR/B scaling)
    B, H, W = 16, 256, 256
    c, p, h = _case(range(100, 116), H, W)
    gp, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c))
    gp = gp.cpu().numpy()
    ref = orc.le_grad_probs(h.astype(np.float64), c.astype(np.float64))
    for b in range(B):
        err = np.abs(gp[b] - ref[b]).max() / np.abs(ref[b]).max()
        assert err <= 1e-4, (b, err)


def test_as_gradient_matches_oracle_and_fd(orc):
    Bg, Hg, Wg = 2, 64, 80  # 4 patches, a 16-column remainder
    pg = np.random.default_rng(5).uniform(0.05, 0.95, size=(Bg, Hg, Wg)).astype(np.float32)
    c, p, h = _case([1], 16, 16)
    prm = hb.default_loss_params()
    _, gg = hb.halftone_loss_backward(to_dev(h), to_dev(c), probs_gray=to_dev(pg), prm=prm)
    gg = gg.cpu().numpy()
    L, ref = orc.as_loss(pg.astype(np.float64))
    ref = prm.w_a * ref
    assert np.abs(gg - ref).max() <= 1e-4 * np.abs(ref).max()
    assert np.all(gg[:, :, 64:] == 0.0)
    # FP64 central differences of the oracle's L_AS at a few pixels
    x = pg.astype(np.float64)
    for (b, y, xx) in [(0, 3, 4), (1, 40, 60), (0, 63, 31)]:
        e = 1e-5
        xp = x.copy(); xp[b, y, xx] += e
        xm = x.copy(); xm[b, y, xx] -= e
        fd = prm.w_a * (orc.as_loss(xp, grad=False)[0] - orc.as_loss(xm, grad=False)[0]) / (2 * e)
        assert abs(gg[b, y, xx] - fd) <= 1e-4 * np.abs(ref).max()


def test_loss_backward_is_deterministic(orc):
    c, p, h = _case([9, 10], 64, 64)
    a, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c))
    b, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c))
    assert torch.equal(a, b)


@pytest.mark.parametrize("prm", [dict(), dict(w_s=1.0)])
def test_coma_gradient_matches_oracle(orc, prm):
    """The COMA estimator (Eqs. baseline, coma) in both gradient spaces."""
    B, H, W = 3, 48, 61
    c, p, h = _case([41, 42, 43], H, W, pseed=4)
    ref = orc.coma_grad_logits(h.astype(np.float64), c.astype(np.float64),
                               p.astype(np.float64), dict(prm, estimator=1))
    lp = hb.default_loss_params(estimator=hb.HS_EST_COMA, **prm)
    gl, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c), to_dev(p), prm=lp,
                                      grad_space=hb.HS_WRT_LOGIT)
    assert np.abs(gl.cpu().numpy() - ref).max() <= 1e-4 * np.abs(ref).max()
    gp, _ = hb.halftone_loss_backward(to_dev(h), to_dev(c), to_dev(p), prm=lp,
                                      grad_space=hb.HS_WRT_PROB)
    refp = ref / (p.astype(np.float64) * (1 - p.astype(np.float64)))
    assert np.abs(gp.cpu().numpy() - refp).max() <= 1e-4 * np.abs(refp).max()


def test_coma_needs_probs():
    c, p, h = _case([44], 16, 16)
    lp = hb.default_loss_params(estimator=hb.HS_EST_COMA)
    with pytest.raises(hb.HalftoneError):
        hb.halftone_loss_backward(to_dev(h), to_dev(c), None, prm=lp)


def test_loss_backward_into_caller_buffers():
    """The binding's caller-provided outputs and workspace (as a training
    loop holds them) give the same gradients as fresh allocations, twice in
    a row on the same buffers."""
    B, H, W = 2, 40, 56
    c, p, h = _case([41, 42], H, W)
    ct, pt, ht = to_dev(c), to_dev(p), to_dev(h)
    ref = hb.halftone_loss_backward(ht, ct, probs=pt, probs_gray=pt, grad_space=hb.HS_WRT_LOGIT)
    out = (torch.full_like(pt, float("nan")), torch.full_like(pt, float("nan")))
    need = hb.lib().halftone_loss_workspace_size(B, H, W, B, H, W,
                                                  ctypes.byref(hb.default_loss_params()))
    ws = torch.empty(need, dtype=torch.uint8, device=ct.device)
    for _ in range(2):
        got = hb.halftone_loss_backward(ht, ct, probs=pt, probs_gray=pt,
                                        grad_space=hb.HS_WRT_LOGIT, workspace=ws, out=out)
        assert got[0].data_ptr() == out[0].data_ptr() and got[1].data_ptr() == out[1].data_ptr()
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    with pytest.raises(AssertionError):
        hb.halftone_loss_backward(ht, ct, probs=pt, probs_gray=pt, out=(out[0][:1], out[1]))
