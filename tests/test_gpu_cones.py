"""GPU tests of the recheck stages after a BF16 pass (the exact bits of
Algorithm 1's TEST threshold): the FP16 cone stage, the split stage behind
it, and their hand-over when FP16's range is exceeded.

Exactness does not depend on the middle stage: every pixel is either
decided by a stage whose error is below that stage's band, or passed on. So
the tests check each stage's error on every pixel, and check that cones
whose FP16 activations (or weights) overflow are passed on, with bits that
still equal the oracle's off the margin."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import inputs, parity_mask, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb

pytestmark = pytest.mark.gpu

# offsets in the flat weight array (W[cout][cin][3][3] then bias per layer)
W2 = 32 * 2 * 9 + 32
L32 = 32 * 32 * 9 + 32


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_logits(orc, w, c, seeds):
    B, H, W = c.shape
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    return orc.policy_forward(w.astype(np.float64), c.astype(np.float64), z)


def _scaled(w, e):
    """Layer 1's weights times 2^e. The He policy has zero biases, so every
    activation and the logit scale by 2^e exactly (ReLU commutes with a
    positive scale; powers of two are exact in FP32 and BF16): the bits and
    the lists of a call with recheck_tau scaled by 2^e are the unscaled
    call's, while FP16 activations (e = 14) or weights (e = 16) overflow."""
    assert np.abs(w[576:576 + 32]).max() == 0.0 and np.all(w[W2 + 9216:W2 + L32] == 0.0)
    w = w.copy()
    w[:576] *= np.float32(2.0 ** e)
    return w


@pytest.mark.parametrize("shape", [(2, 64, 90), (1, 13, 300)])
def test_fp16_cone_stage_on_every_pixel(orc, shape):
    # every pixel listed and decided by the FP16 stage (a band of 1e-30):
    # its logits must be within a fraction of the BF16 pass's error of the
    # oracle's, and the bits off its own band must be the oracle's
    B, H, W = shape
    seeds = list(range(301, 301 + B))
    _say("fp16 cones on every pixel", shape)
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds)
    pol = hb.Policy(to_dev(w))
    ct, st = to_dev(c), seeds_t(seeds)
    bits, lg, stt = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_BF16,
                                             recheck_tau=1e30, recheck_tau16=1e-30,
                                             recheck_tau2=0.0, logits=True, stats=True)
    stt, lg, bits = stt.cpu().numpy(), lg.cpu().numpy(), bits.cpu().numpy()
    assert stt[0] == B * H * W
    assert stt[4] <= 2  # only exact zeros go on
    err16 = np.abs(lg - ref).max()
    _, l16 = hb.halftone_infer(to_dev(w), ct, st, precision=hb.HS_BF16, recheck_tau=0.0,
                               logits=True)
    errb = np.abs(l16.cpu().numpy() - ref).max()
    _say("fp16 cone error", err16, "bf16 pass error", errb)
    assert 0.0 < err16 < errb / 3
    off = np.abs(ref) > 2 * err16
    assert np.array_equal(bits[off], (ref >= 0)[off].astype(np.uint8))


def test_fp16_stage_keeps_the_bits_and_splits_the_work(orc):
    B, H, W = 2, 200, 256
    seeds = [311, 312]
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds)
    tau = 0.055
    pol = hb.Policy(to_dev(w))
    bits, stt = hb.halftone_policy_infer(pol, to_dev(c), seeds_t(seeds), precision=hb.HS_BF16,
                                         recheck_tau=tau, recheck_tau16=tau / 4, stats=True)
    stt, bits = stt.cpu().numpy(), bits.cpu().numpy()
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    # the FP16 stage decides most listed pixels: about 3/4 at tau16 = tau / 4
    _say("listed", stt[0], "to split", stt[4], "to fp32", stt[2])
    assert 0 < stt[4] < 0.5 * stt[0]
    assert 0 <= stt[2] <= stt[4]
    # without the stage (the default) the split stage takes every listed pixel
    _, st0 = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), precision=hb.HS_BF16,
                               recheck_tau=tau, stats=True)
    st0 = st0.cpu().numpy()
    assert st0[0] == stt[0] and st0[4] == st0[0]


@pytest.mark.parametrize("e", [14, 16])
def test_fp16_overflow_passes_cones_on(orc, e):
    # e = 14: activations beyond FP16's range in most cones (the He policy's
    # activations reach about 8, and 4 x 2^14 > 65504); e = 16: layer-1
    # weights themselves beyond it (then every cone goes on)
    B, H, W = 2, 64, 96
    seeds = [321, 322]
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds)
    ws = _scaled(w, e)
    assert (np.abs(ws[:576]).max() >= 65520) == (e == 16)
    ct, st = to_dev(c), seeds_t(seeds)
    tau = 0.055
    _say("fp16 overflow", e)
    b0, s0 = hb.halftone_policy_infer(hb.Policy(to_dev(w)), ct, st, precision=hb.HS_BF16,
                                      recheck_tau=tau, recheck_tau16=tau / 4, stats=True)
    b1, s1 = hb.halftone_policy_infer(hb.Policy(to_dev(ws)), ct, st, precision=hb.HS_BF16,
                                      recheck_tau=tau * 2.0 ** e,
                                      recheck_tau16=tau * 2.0 ** e / 4, stats=True)
    s0, s1 = s0.cpu().numpy(), s1.cpu().numpy()
    _say("unscaled", s0, "scaled", s1)
    assert s1[0] == s0[0]  # the BF16 pass lists the same pixels
    assert s1[4] > s0[4]   # overflowed cones went on to the split stage
    if e == 16:
        assert s1[4] == s1[0]
    m = parity_mask(orc, ref)
    for b in (b0, b1):
        b = b.cpu().numpy()
        assert np.array_equal(b[m], (ref >= 0)[m].astype(np.uint8))
    # packed again from the same weights: the same flags and results
    pol = hb.Policy(to_dev(ws))
    b2, s2 = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_BF16,
                                      recheck_tau=tau * 2.0 ** e,
                                      recheck_tau16=tau * 2.0 ** e / 4, stats=True)
    assert torch.equal(b2, b1) and np.array_equal(s2.cpu().numpy(), s1)


def test_fp16_stage_with_levels(orc):
    # multitone levels: the stage decides the distance to the nearest
    # threshold the same way
    shapes = [(70, 90), (33, 140)]
    seeds = [331, 332]
    from paper_2304_12152_amd import synth
    w = synth.he_weights(42)
    cs = [synth.contone(s, h, ww) for s, (h, ww) in zip(seeds, shapes)]
    c = np.concatenate([x.ravel() for x in cs])
    out, stt = hb.halftone_policy_infer(hb.Policy(to_dev(w)), to_dev(c), seeds_t(seeds), shapes,
                                        precision=hb.HS_BF16, recheck_tau=0.055,
                                        recheck_tau16=0.055 / 4, stats=True, levels=4)
    out, stt = out.cpu().numpy(), stt.cpu().numpy()
    assert stt[0] > 0 and 0 < stt[4] < stt[0]
    off = 0
    thr = np.log((2.0 * np.arange(3) + 1.0) / (2.0 * 4 - 3.0 - 2.0 * np.arange(3)))
    for s, (h, ww), cc in zip(seeds, shapes, cs):
        ref = _oracle_logits(orc, w, cc[None], [s])[0]
        lev = (ref[..., None] >= thr).sum(-1)
        dist = np.abs(ref[..., None] - thr).min(-1)
        keep = dist > 4e-4
        got = out[off:off + h * ww].reshape(h, ww)
        assert np.array_equal(got[keep], lev[keep])
        off += h * ww
