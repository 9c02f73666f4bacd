"""GPU parity of the FP16 inference pass (precision HS_FP16) against the
oracle: FP16 carries three more mantissa bits than BF16 at the same matrix
core rate, so its recheck band is about 8 times narrower; the bits must
still equal the oracle's wherever |p - 0.5| > 1e-4. An activation beyond
FP16's range sends the whole pass through BF16 again, on the device."""
import sys

import numpy as np
import pytest

from gpu_common import inputs, parity_mask, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb

pytestmark = pytest.mark.gpu

TAU16 = hb.RECHECK_TAU[hb.HS_FP16]
SHAPES = [(1, 1, 1), (1, 3, 200), (1, 37, 45), (2, 64, 130), (1, 256, 256)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_logits(orc, w, c, seeds):
    B, H, W = c.shape
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    return orc.policy_forward(w.astype(np.float64), c.astype(np.float64), z)


@pytest.mark.parametrize("shape", SHAPES)
def test_fp16_with_recheck_matches_oracle(orc, shape):
    B, H, W = shape
    seeds = list(range(21, 21 + B))
    _say("infer fp16", shape)
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds)
    bits, lg, st = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_FP16,
                                     logits=True, stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    near = np.abs(lg) < TAU16
    assert np.abs(lg[near] - ref[near]).max(initial=0.0) <= 5e-4
    nearer = np.abs(lg) < 1.5e-4  # tau2 = max(tau / 64, 1.5e-4)
    assert np.abs(lg[nearer] - ref[nearer]).max(initial=0.0) <= 2e-5 * max(1.0, np.abs(ref).max())
    assert np.abs(lg - ref).max() < TAU16
    assert st[0] >= near.sum() and 0 <= st[1] <= st[0] and 0 <= st[2] <= st[0]
    assert st[3] == 0


def test_fp16_c2_error_and_bits():
    """8 x 1024 x 1024: the raw FP16 logits (recheck_tau = 0, nothing
    listed) stay within tau / 1.25 of the FP32 path's, and with the default
    band the bits equal FP32's wherever |x_fp32| > 4.1e-4."""
    B, H, W = 8, 1024, 1024
    seeds = list(range(101, 109))
    _say("infer fp16 C2")
    w, c = inputs(seeds, H, W)
    wt, ct, st = to_dev(w), to_dev(c), seeds_t(seeds)
    b32, l32 = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP32, logits=True)
    _, raw = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP16, 0.0, logits=True)
    _, rawb = hb.halftone_infer(wt, ct, st, 0, hb.HS_BF16, 0.0, logits=True)
    err16 = float((raw - l32).abs().max())
    err_bf = float((rawb - l32).abs().max())
    _say("max |logit error|: fp16 %.5f bf16 %.5f" % (err16, err_bf))
    assert err16 < TAU16 / 1.25 and err16 < err_bf / 4
    b16, stats = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP16, stats=True)
    b32, l32, b16 = b32.cpu().numpy(), l32.cpu().numpy(), b16.cpu().numpy()
    m = np.abs(l32) > 4.1e-4
    assert np.array_equal(b16[m], b32[m])
    stats = stats.cpu().numpy()
    _say("fp16 stats", stats.tolist())
    assert stats[3] == 0 and stats[0] > 0


def _scaled(w, s):
    """Layer 1 (weights and bias) times s, layer 2's weights divided by s:
    ReLU commutes with a positive scale, so the network is the same, but the
    layer-1 activations grow by s."""
    w = w.copy()
    n1 = 32 * 2 * 9
    w[:n1 + 32] *= s
    w[n1 + 32:n1 + 32 + 32 * 32 * 9] /= s
    return w


def test_fp16_overflow_reruns_in_bf16(orc):
    """With layer-1 activations scaled by 2^16 the FP16 pass overflows; the
    call then decides every pixel from the BF16 pass with an 8 times wider
    band. Power-of-two scaling is exact in BF16 and FP32, so the result
    equals the unscaled network's BF16 result bit for bit, except that the
    split stage keeps the FP16 call's tau2 (max(tau / 64, 1.5e-4)),
    so pixels between the two tau2 are decided by different stages."""
    B, H, W = 2, 40, 150
    seeds = [41, 42]
    _say("infer fp16 overflow re-run")
    w, c = inputs(seeds, H, W)
    ws = _scaled(w, 2.0 ** 16)
    assert hb.HS_PARAM_COUNT == w.size
    ct, st = to_dev(c), seeds_t(seeds)
    bits, lg, stats = hb.halftone_infer(to_dev(ws), ct, st, 0, hb.HS_FP16, logits=True,
                                        stats=True)
    # the reference: a BF16 call with the 8 times wider band and, as after
    # an FP16 pass, without the FP16 cone stage (tau16 = 0)
    ref_bits, ref_lg, ref_stats = hb.halftone_policy_infer(
        hb.Policy(to_dev(w)), ct, st, precision=hb.HS_BF16, recheck_tau=8 * TAU16,
        recheck_tau16=0.0, logits=True, stats=True)
    stats, ref_stats = stats.cpu().numpy(), ref_stats.cpu().numpy()
    assert stats[3] == 1 and ref_stats[3] == 0
    assert stats[0] == ref_stats[0]  # the same BF16 list (band 8 tau)
    lg, ref_lg = lg.cpu().numpy(), ref_lg.cpu().numpy()
    same = np.abs(ref_lg) >= max(8 * TAU16 / 64, 1.5e-4)  # the larger tau2
    assert np.array_equal(bits.cpu().numpy()[same], ref_bits.cpu().numpy()[same])
    assert np.array_equal(lg[same], ref_lg[same])
    assert np.abs(lg - ref_lg).max() <= 5e-4
    ref = _oracle_logits(orc, w, c, seeds)
    m = parity_mask(orc, ref)
    assert np.array_equal(bits.cpu().numpy()[m], (ref >= 0)[m].astype(np.uint8))
    # the same weights without the scale stay in range
    _, st2 = hb.halftone_infer(to_dev(w), ct, st, 0, hb.HS_FP16, stats=True)
    assert st2.cpu().numpy()[3] == 0


def test_fp16_form_that_tests_every_layer(orc):
    """Layer 1 scaled by 2^12 (layer 2 by 2^-12): its a priori bound passes
    FP16's range, so the form that tests every layer runs; its activations
    (at most a few times 2^12) still fit, so it decides, to the oracle."""
    B, H, W = 1, 64, 130
    seeds = [61]
    _say("infer fp16, every layer tested")
    w, c = inputs(seeds, H, W)
    ws = _scaled(w, 2.0 ** 12)
    ref = _oracle_logits(orc, ws, c, seeds)
    bits, lg, st = hb.halftone_infer(to_dev(ws), to_dev(c), seeds_t(seeds), 0, hb.HS_FP16,
                                     logits=True, stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    assert st[3] == 0
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    assert np.abs(lg - ref).max() < TAU16


def test_fp16_contone_outside_the_unit_range_reruns_in_bf16():
    """The layer bounds assume contones in [0, 1]; a page with values
    outside is decided by the BF16 pass, bit for bit as a BF16 call with
    the 8 times wider band wherever both calls' split stages decide."""
    B, H, W = 2, 50, 90
    seeds = [71, 72]
    _say("infer fp16, contone outside [0, 1]")
    w, c = inputs(seeds, H, W)
    for bad in (1.25, -0.5):
        cb = c.copy()
        cb[1, 20, 33] = bad
        ct, st = to_dev(cb), seeds_t(seeds)
        bits, lg, stats = hb.halftone_infer(to_dev(w), ct, st, 0, hb.HS_FP16, logits=True,
                                            stats=True)
        rb, rl = hb.halftone_policy_infer(hb.Policy(to_dev(w)), ct, st, precision=hb.HS_BF16,
                                          recheck_tau=8 * TAU16, recheck_tau16=0.0, logits=True)
        assert stats.cpu().numpy()[3] == 1, bad
        lg, rl = lg.cpu().numpy(), rl.cpu().numpy()
        same = np.abs(rl) >= max(8 * TAU16 / 64, 1.5e-4)  # split-stage decisions in both
        assert np.array_equal(bits.cpu().numpy()[same], rb.cpu().numpy()[same])
        assert np.array_equal(lg[same], rl[same])
        assert np.abs(lg - rl).max() <= 5e-4


def test_fp16_pages_and_levels(orc):
    """Uneven pages in one launch, binary and with 4 levels."""
    pages = [(37, 200), (130, 129), (5, 300)]
    seeds = [51, 52, 53]
    _say("infer fp16 pages")
    w = inputs([0], 1, 1)[0]
    from paper_2304_12152_amd import synth
    cs = [synth.contone_batch([s], h, ww)[0] for s, (h, ww) in zip(seeds, pages)]
    flat = np.concatenate([x.ravel() for x in cs]).astype(np.float32)
    for levels in (None, 4):
        out, lg = hb.halftone_infer_pages(to_dev(w), to_dev(flat), seeds_t(seeds), pages,
                                          precision=hb.HS_FP16, logits=True, levels=levels)
        ref32, lg32 = hb.halftone_infer_pages(to_dev(w), to_dev(flat), seeds_t(seeds), pages,
                                              precision=hb.HS_FP32, logits=True, levels=levels)
        out, lg, ref32, lg32 = (t.cpu().numpy() for t in (out, lg, ref32, lg32))
        L = 2 if levels is None else levels
        thr = np.log((2 * np.arange(L - 1) + 1) / (2 * L - 3 - 2 * np.arange(L - 1)))
        dist = np.min(np.abs(lg32[:, None] - thr[None, :]), axis=1)
        m = dist > 4.1e-4
        assert np.array_equal(out[m], ref32[m]), levels
        assert np.abs(lg - lg32).max() < TAU16
    # the binary pages against the oracle, page by page
    off = 0
    for s, (h, ww), x in zip(seeds, pages, cs):
        ref = _oracle_logits(orc, w, x[None], [s])[0]
        o = hb.halftone_infer_pages(to_dev(w), to_dev(flat), seeds_t(seeds), pages,
                                    precision=hb.HS_FP16).cpu().numpy()[off:off + h * ww]
        m = parity_mask(orc, ref).ravel()
        assert np.array_equal(o[m], (ref.ravel() >= 0)[m].astype(np.uint8))
        off += h * ww


def test_fp16_overflow_reruns_in_bf16_with_levels(orc):
    """The same re-run for the multitoning call (4 levels): the FP16 pass of
    the 2^16-scaled network overflows, and the levels equal a BF16 call's on
    the unscaled network wherever both calls' split stages decide."""
    pages = [(40, 150), (33, 70)]
    seeds = [81, 82]
    _say("infer fp16 overflow re-run, 4 levels")
    w = inputs([0], 1, 1)[0]
    from paper_2304_12152_amd import synth
    flat = np.concatenate([synth.contone_batch([s], h, ww)[0].ravel()
                           for s, (h, ww) in zip(seeds, pages)]).astype(np.float32)
    ft, st = to_dev(flat), seeds_t(seeds)
    out, lg, stats = hb.halftone_infer_pages(to_dev(_scaled(w, 2.0 ** 16)), ft, st, pages,
                                             precision=hb.HS_FP16, logits=True, stats=True,
                                             levels=4)
    ref, rl, rst = hb.halftone_policy_infer(hb.Policy(to_dev(w)), ft, st, pages,
                                            precision=hb.HS_BF16, recheck_tau=8 * TAU16,
                                            recheck_tau16=0.0, logits=True, stats=True, levels=4)
    stats, rst = stats.cpu().numpy(), rst.cpu().numpy()
    assert stats[3] == 1 and rst[3] == 0 and stats[0] == rst[0]
    lg, rl = lg.cpu().numpy(), rl.cpu().numpy()
    thr = np.log(np.array([1.0, 3.0, 5.0]) / np.array([5.0, 3.0, 1.0]))
    dist = np.min(np.abs(rl[:, None] - thr[None, :]), axis=1)
    same = dist >= max(8 * TAU16 / 64, 1.5e-4)
    assert np.array_equal(out.cpu().numpy()[same], ref.cpu().numpy()[same])
    assert np.array_equal(lg[same], rl[same])
