"""GPU parity of the FP8 inference pass (precision HS_FP8 on a packed policy
with its FP8 copy) against the oracle. The four 32->32 convolutions run on
the FP8 E4M3 matrix cores with per-output-channel weight scales and
per-layer activation scales (calibrated on images other than the ones
checked); E4M3 keeps 4 significant bits to BF16's 8, so the logit error and
the recheck band are an order of magnitude wider, and the bits must still
equal the oracle's wherever |p - 0.5| > 1e-4. An activation beyond the
calibrated range saturates E4M3 and sends the pass through BF16 again."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import inputs, oracle_threads, parity_mask, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import calibrate, synth

pytestmark = pytest.mark.gpu

CAL_SEEDS = [3_300_001, 3_300_002]  # calibration contones (not used below)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_logits(orc, w, c, seeds):
    B, H, W = c.shape
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    with orc.threads(oracle_threads()):
        return orc.policy_forward(w.astype(np.float64), c.astype(np.float64), z)


@pytest.fixture(scope="module")
def he():
    w = inputs([0], 1, 1)[0]
    return w


@pytest.fixture(scope="module")
def cal(he):
    _say("calibrating the FP8 pass of the He policy")
    b = calibrate.bands(to_dev(he), hb.HS_FP8, seeds=CAL_SEEDS)
    _say("fp8 bands", {k: v for k, v in b.items() if k not in ("errors", "policy")},
         b["errors"], "act_max", b["policy"].act_max.tolist())
    return b


def test_layer_max_matches_the_oracle(orc, he):
    """halftone_layer_max: per layer, the largest activation of the FP32
    forward. The oracle's network ends in one output channel without a
    ReLU, so channel c of layer k is read out through a stack of k hidden
    layers and a last layer whose only weight is 1 at (c, centre tap)."""
    B, H, W = 2, 23, 41
    seeds = [3_300_101, 3_300_102]
    c = synth.contone_batch(seeds, H, W)
    got = hb.halftone_layer_max(to_dev(he), to_dev(c), seeds_t(seeds)).cpu().numpy()
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    nw = [2 * 32 * 9 + 32] + [32 * 32 * 9 + 32] * 4  # parameters of layers 1..5
    for k in range(1, 6):
        ch = (2,) + (32,) * k + (1,)
        body = he[:sum(nw[:k])].astype(np.float64)
        ref = 0.0
        for cc in range(32):
            last = np.zeros(32 * 9 + 1)
            last[cc * 9 + 4] = 1.0
            x = orc.policy_forward(np.concatenate([body, last]), c.astype(np.float64), z, ch=ch)
            ref = max(ref, float(x.max()))
        _say("layer", k, "max", got[k - 1], "oracle", ref)
        assert abs(got[k - 1] - ref) <= 1e-5 * ref


def test_fp8_pass_error_and_scales(cal, he):
    """The FP8 pass's raw logits (recheck_tau = 0) on images other than the
    calibration ones stay within the band / 1.5 of FP32's; the scales leave
    the calibration maxima 4 to 8 times below E4M3's 448."""
    pol = cal["policy"]
    a = pol.act_max
    s = 2.0 ** np.ceil(np.log2(4 * a / 448.0))
    assert np.all(4 * a <= 448 * s) and np.all(8 * a > 448 * s)
    seeds = [3_300_011, 3_300_012]
    c = synth.contone_batch(seeds, 384, 384)
    wt, ct, st = to_dev(he), to_dev(c), seeds_t(seeds)
    _, l32 = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP32, logits=True)
    _, l8, stt = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_FP8, recheck_tau=0.0,
                                          logits=True, stats=True)
    _, lb = hb.halftone_infer(wt, ct, st, 0, hb.HS_BF16, 0.0, logits=True)
    e8 = float((l8 - l32).abs().max())
    eb = float((lb - l32).abs().max())
    _say("max |logit error|: fp8 %.4f bf16 %.4f (band %.4f)" % (e8, eb, cal["tau"]))
    assert int(stt[3]) == 0
    assert e8 < cal["tau"] / 1.5 * 1.2  # the calibration margin, less 20% for new images
    assert e8 > 2 * eb  # FP8 really ran: its error is well above BF16's


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 3, 200), (1, 37, 45), (2, 64, 130),
                                   (1, 256, 256)])
def test_fp8_with_recheck_matches_oracle(orc, cal, he, shape):
    B, H, W = shape
    seeds = list(range(3_300_021, 3_300_021 + B))
    _say("infer fp8", shape)
    c = synth.contone_batch(seeds, H, W)
    ref = _oracle_logits(orc, he, c, seeds)
    bits, lg, st = hb.halftone_policy_infer(cal["policy"], to_dev(c), seeds_t(seeds),
                                            precision=hb.HS_FP8, recheck_tau=cal["tau"],
                                            recheck_tau2=cal["tau2"], logits=True, stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    assert np.abs(lg - ref).max() < cal["tau"]
    near = np.abs(lg) < cal["tau"]  # decided by the split stage
    assert np.abs(lg[near] - ref[near]).max(initial=0.0) <= cal["tau2"]
    assert st[3] == 0 and st[0] >= near.sum() and st[4] == st[0]


def _scaled(w, s):
    """Layer 1 (weights and bias) times s, layer 2's weights divided by s:
    the same network, with layer-1 activations s times larger."""
    w = w.copy()
    n1 = 32 * 2 * 9
    w[:n1 + 32] *= s
    w[n1 + 32:n1 + 32 + 32 * 32 * 9] /= s
    return w


def test_fp8_saturation_reruns_in_bf16(orc, cal, he):
    """A policy whose FP8 copy was scaled for the unscaled network but whose
    layer-1 activations are 64 times larger saturates E4M3; the pass then
    runs again in BF16 with tau / 8, decided on the device, and the bits
    still equal the oracle's."""
    B, H, W = 2, 40, 150
    seeds = [3_300_041, 3_300_042]
    c = synth.contone_batch(seeds, H, W)
    ws = _scaled(he, 64.0)
    pol = hb.Policy(to_dev(ws)).set_fp8(cal["policy"].act_max)  # layer 1's max 64 x too small
    ct, st = to_dev(c), seeds_t(seeds)
    bits, lg, stats = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_FP8,
                                               recheck_tau=cal["tau"], recheck_tau2=cal["tau2"],
                                               logits=True, stats=True)
    stats = stats.cpu().numpy()
    _say("saturated fp8 stats", stats.tolist())
    assert stats[3] == 1
    # the BF16 re-run lists what a BF16 call with tau / 8 lists
    _, rst = hb.halftone_policy_infer(hb.Policy(to_dev(ws)), ct, st, precision=hb.HS_BF16,
                                      recheck_tau=cal["tau"] / 8, recheck_tau16=0.0,
                                      recheck_tau2=cal["tau2"], stats=True)
    assert stats[0] == int(rst.cpu().numpy()[0])
    ref = _oracle_logits(orc, he, c, seeds)
    m = parity_mask(orc, ref)
    assert np.array_equal(bits.cpu().numpy()[m], (ref >= 0)[m].astype(np.uint8))
    # the unscaled weights with the same scales do not saturate
    _, s2 = hb.halftone_policy_infer(cal["policy"], ct, st, precision=hb.HS_FP8,
                                     recheck_tau=cal["tau"], stats=True)
    assert s2.cpu().numpy()[3] == 0


def test_fp8_pages_and_levels(orc, cal, he):
    """Uneven pages in one launch, binary and with 4 levels, against the
    FP32 path off the margin, and the binary pages against the oracle."""
    pages = [(37, 200), (130, 129), (5, 300)]
    seeds = [3_300_051, 3_300_052, 3_300_053]
    cs = [synth.contone_batch([s], h, ww)[0] for s, (h, ww) in zip(seeds, pages)]
    flat = np.concatenate([x.ravel() for x in cs]).astype(np.float32)
    wt, ft, st = to_dev(he), to_dev(flat), seeds_t(seeds)
    for levels in (2, 4):
        out, lg = hb.halftone_policy_infer(cal["policy"], ft, st, pages, precision=hb.HS_FP8,
                                           recheck_tau=cal["tau"], recheck_tau2=cal["tau2"],
                                           logits=True, levels=levels)
        ref32, lg32 = hb.halftone_infer_pages(wt, ft, st, pages, precision=hb.HS_FP32,
                                              logits=True, levels=levels)
        out, lg, ref32, lg32 = (t.cpu().numpy() for t in (out, lg, ref32, lg32))
        thr = np.log((2 * np.arange(levels - 1) + 1) / (2 * levels - 3 - 2 * np.arange(levels - 1)))
        dist = np.min(np.abs(lg32[:, None] - thr[None, :]), axis=1)
        m = dist > 4.1e-4
        assert np.array_equal(out[m], ref32[m]), levels
        assert np.abs(lg - lg32).max() < cal["tau"]
        if levels == 2:
            off = 0
            for s, (h, ww), x in zip(seeds, pages, cs):
                ref = _oracle_logits(orc, he, x[None], [s])[0]
                mo = parity_mask(orc, ref).ravel()
                o = out[off:off + h * ww]
                assert np.array_equal(o[mo], (ref.ravel() >= 0)[mo].astype(np.uint8))
                off += h * ww


def test_fp8_needs_its_copy(he):
    """HS_FP8 is refused by the unpacked calls and by a policy without its
    FP8 copy; packing again clears the copy."""
    c = synth.contone_batch([3_300_061], 16, 16)
    wt, ct, st = to_dev(he), to_dev(c), seeds_t([3_300_061])
    with pytest.raises(hb.HalftoneError) as e:
        hb.halftone_infer(wt, ct, st, 0, hb.HS_FP8, 1.0)
    assert e.value.code == hb.HS_EUNSUPPORTED
    pol = hb.Policy(wt)
    with pytest.raises(hb.HalftoneError) as e:
        hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_FP8, recheck_tau=1.0)
    assert e.value.code == hb.HS_EUNSUPPORTED
    with pytest.raises(hb.HalftoneError) as e:
        pol.set_fp8([1.0, float("nan"), 1.0, 1.0])
    assert e.value.code == hb.HS_EINVAL
    pol.set_fp8([1.0, 1.0, 1.0, 1.0])
    assert pol.handle.fp8 == 1
    hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_FP8, recheck_tau=1.0)


def test_fp8_c2_full_size_sampled(orc, cal, he):
    """8 x 1024 x 1024 in the bench's launch: bits equal the FP32 path's
    wherever |x_fp32| > 4.1e-4, and the oracle's on sampled windows."""
    B, H, W = 8, 1024, 1024
    seeds = list(range(101, 109))
    c = synth.contone_batch(seeds, H, W)
    wt, ct, st = to_dev(he), to_dev(c), seeds_t(seeds)
    _say("infer fp8 C2")
    b8, stats = hb.halftone_policy_infer(cal["policy"], ct, st, precision=hb.HS_FP8,
                                         recheck_tau=cal["tau"], recheck_tau2=cal["tau2"],
                                         stats=True)
    b32, l32 = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP32, logits=True)
    stats = stats.cpu().numpy()
    _say("fp8 C2 stats", stats.tolist())
    m = (l32.abs() > 4.1e-4)
    assert int(((b8 != b32) & m).sum()) == 0
    assert stats[3] == 0
    b8 = b8.cpu().numpy()
    rng = np.random.default_rng(7)
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    for _ in range(6):
        b = int(rng.integers(B))
        y0, x0 = int(rng.integers(0, H - 24)), int(rng.integers(0, W - 24))
        ref = orc.policy_forward_window(he.astype(np.float64), c[b].astype(np.float64), z[b],
                                        y0, y0 + 24, x0, x0 + 24)
        mo = parity_mask(orc, ref)
        assert np.array_equal(b8[b, y0:y0 + 24, x0:x0 + 24][mo], (ref >= 0)[mo].astype(np.uint8))
