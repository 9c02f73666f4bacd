"""GPU parity of halftone_infer (Algorithm 1, TEST) against the oracle.

Bits must equal the oracle's wherever |p - 0.5| > 1e-4 (FP32 and BF16 with
the FP32 recheck); FP32 logits must agree to FP32 rounding."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import P_MARGIN, device, inputs, parity_mask, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 3, 200), (1, 37, 45), (2, 64, 130), (1, 256, 256)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_logits(orc, w, c, seeds, kind):
    B, H, W = c.shape
    z = orc.noise_map(seeds, H, W, kind=kind, stream=1, step=0)
    return orc.policy_forward(w.astype(np.float64), c.astype(np.float64), z)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", [hb.HS_NOISE_UNIFORM, hb.HS_NOISE_GAUSS])
def test_fp32_matches_oracle(orc, shape, kind):
    B, H, W = shape
    seeds = list(range(11, 11 + B))
    _say("infer fp32", shape, kind)
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds, kind)
    bits, lg = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), kind, hb.HS_FP32,
                                 logits=True)
    lg = lg.cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(lg - ref).max() <= 2e-5 * scale
    m = parity_mask(orc, ref)
    assert np.array_equal(bits.cpu().numpy()[m], (ref >= 0)[m].astype(np.uint8))


@pytest.mark.parametrize("shape", SHAPES)
def test_bf16_with_recheck_matches_oracle(orc, shape):
    B, H, W = shape
    seeds = list(range(21, 21 + B))
    _say("infer bf16", shape)
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds, 0)
    tau = 0.055
    bits, lg, st = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_BF16, tau,
                                     logits=True, stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    # rechecked pixels carry the FP16 cone stage's logit (about 1/8 of the
    # BF16 error) or, within tau16 = tau / 4 of the threshold, the split-BF16
    # one (~2^-8 of BF16's) or, within tau2, the FP32 one; the others a BF16
    # logit
    near = np.abs(lg) < tau
    assert np.abs(lg[near] - ref[near]).max(initial=0.0) <= tau / 8
    near16 = np.abs(lg) < tau / 4
    assert np.abs(lg[near16] - ref[near16]).max(initial=0.0) <= 5e-4
    tau2 = max(tau / 64, 1.5e-4)
    nearer = np.abs(lg) < tau2
    assert np.abs(lg[nearer] - ref[nearer]).max(initial=0.0) <= 2e-5 * max(1.0, np.abs(ref).max())
    assert np.abs(lg - ref).max() < tau
    assert st[0] >= near.sum() and 0 <= st[1] <= st[0] and 0 <= st[2] <= st[0]


@pytest.mark.parametrize("shape", [(3, 50, 70), (1, 13, 300)])
def test_split_stage_on_every_pixel(orc, shape):
    """recheck_tau above every |x|: every pixel goes through the split-BF16
    cone pipeline (thousands of two-cone batches per launch, cones at every
    border); each logit it returns must be within the split error of the
    oracle's, and those it hands to the FP32 stage (an explicit tau2 of a
    packed policy) within FP32 rounding."""
    B, H, W = shape
    seeds = list(range(31, 31 + B))
    _say("infer split stage on every pixel", shape)
    w, c = inputs(seeds, H, W)
    ref = _oracle_logits(orc, w, c, seeds, 0)
    tau, tau2 = 1e9, 1e-2
    pol = hb.Policy(to_dev(w))
    bits, lg, st = hb.halftone_policy_infer(pol, to_dev(c), seeds_t(seeds), precision=hb.HS_BF16,
                                            recheck_tau=tau, recheck_tau2=tau2, logits=True,
                                            stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    assert st[0] == B * H * W
    assert np.abs(lg - ref).max() <= 5e-4
    nearer = np.abs(lg) < tau2
    assert np.abs(lg[nearer] - ref[nearer]).max(initial=0.0) <= 2e-5 * max(1.0, np.abs(ref).max())
    assert abs(int(st[2]) - int(nearer.sum())) <= 2
    m = parity_mask(orc, ref)
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))
    # the default band rule tau2 = max(tau / 64, 1.5e-4) sends every pixel on
    # to the FP32 stage at this tau
    bits, lg, st = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_BF16, tau,
                                     logits=True, stats=True)
    st = st.cpu().numpy()
    assert st[0] == st[2] == B * H * W
    assert np.abs(lg.cpu().numpy() - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())
    bits = bits.cpu().numpy()
    assert np.array_equal(bits[m], (ref >= 0)[m].astype(np.uint8))


def test_infer_is_deterministic(orc):
    seeds = [5, 6]
    w, c = inputs(seeds, 96, 80)
    a = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_BF16, 0.08)
    b = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_BF16, 0.08)
    assert torch.equal(a, b)


def test_c2_full_size_sampled(orc):
    """8 x 1024 x 1024 (the inference workload): the oracle is evaluated on
    sampled pixels one receptive field at a time; the whole BF16 map is
    checked against the whole FP32 map wherever FP32 is off-margin."""
    B, H, W = 8, 1024, 1024
    seeds = list(range(11, 19))
    _say("infer C2 full size")
    w, c = inputs(seeds, H, W)
    wt, ct, st = to_dev(w), to_dev(c), seeds_t(seeds)
    b32, l32 = hb.halftone_infer(wt, ct, st, 0, hb.HS_FP32, logits=True)
    b16, l16, stats = hb.halftone_infer(wt, ct, st, 0, hb.HS_BF16, 0.055, logits=True, stats=True)
    b32, l32, b16 = b32.cpu().numpy(), l32.cpu().numpy(), b16.cpu().numpy()
    rng = np.random.default_rng(0)
    wd = w.astype(np.float64)
    for b in range(B):
        pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2), (5, 700)]
        pts += [tuple(int(v) for v in p) for p in rng.integers(0, [H, W], size=(12, 2))]
        for (y, x) in pts:
            ref = window_logit(orc, wd, c[b], seeds[b], y, x)
            assert abs(l32[b, y, x] - ref) <= 2e-5 * max(1.0, abs(ref))
            if abs(orc.sigmoid(ref) - 0.5) > P_MARGIN:
                assert b32[b, y, x] == (ref >= 0) and b16[b, y, x] == (ref >= 0)
    m = np.abs(l32) > 4.1e-4
    assert np.array_equal(b16[m], b32[m])
    # the oracle over one 48 x 48 window per image, and on the 200 listed
    # pixels per image nearest the threshold (the ones the recheck stages
    # decide), one receptive field each
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    l16n = l16.cpu().numpy()
    checked = 0
    for b in range(B):
        y0, x0 = int(rng.integers(0, H - 48)), int(rng.integers(0, W - 48))
        ref = orc.policy_forward_window(wd, c[b].astype(np.float64), z[b], y0, y0 + 48, x0, x0 + 48)
        mw = parity_mask(orc, ref)
        assert np.array_equal(b16[b, y0:y0 + 48, x0:x0 + 48][mw], (ref >= 0)[mw].astype(np.uint8))
        listed = np.argwhere(np.abs(l16n[b]) < 0.055)
        order = np.argsort(np.abs(l32[b][listed[:, 0], listed[:, 1]]))[:200]
        for (y, x) in listed[order]:
            r = window_logit(orc, wd, c[b], seeds[b], int(y), int(x))
            if abs(orc.sigmoid(r) - 0.5) > P_MARGIN:
                assert b16[b, y, x] == (r >= 0), (b, y, x, r)
                checked += 1
    _say("C2: listed pixels checked against the oracle off the margin:", checked)
    assert checked > 8 * 100
    # every rechecked logit is the FP16 cone stage's or, nearer the
    # threshold, the split stage's or the FP32 stage's; each agrees with the
    # FP32 path to its error
    l16 = l16.cpu().numpy()
    near = np.abs(l16) < 0.055
    assert int(stats[0]) >= int(near.sum()) > 0
    assert np.abs(l16[near] - l32[near]).max() <= 0.055 / 8
    near16 = np.abs(l16) < 0.055 / 4
    assert np.abs(l16[near16] - l32[near16]).max() <= 5e-4
    nearer = np.abs(l16) < max(0.055 / 64, 1.5e-4)
    assert np.abs(l16[nearer] - l32[nearer]).max() <= 1e-4


def window_logit(orc, wd, cimg, seed, y, x):
    """Oracle logit at (y, x) of an H x W image from its receptive field only.

    The crop [y-6, y+7) x [x-6, x+7), clipped to the image, contains every
    value the 13 x 13 receptive field reads; its edges are either image edges
    (where the zero padding applies in both) or lie outside the field, so the
    crop evaluated as an image gives the full image's logit at (y, x)."""
    H, W = cimg.shape
    y0, y1, x0, x1 = max(0, y - 6), min(H, y + 7), max(0, x - 6), min(W, x + 7)
    zc = np.array([[orc.normal(seed, yy * W + xx, 1, 0) for xx in range(x0, x1)]
                   for yy in range(y0, y1)])
    cc = cimg[y0:y1, x0:x1].astype(np.float64)
    return float(orc.policy_forward_window(wd, cc, zc, y - y0, y - y0 + 1, x - x0,
                                           x - x0 + 1)[0, 0])


PAGES = [(1, 1), (3, 200), (37, 45), (150, 90), (64, 300), (13, 13), (130, 117)]


def _pages_inputs(shapes, seed0):
    w = synth.he_weights(42)
    seeds = [seed0 + i for i in range(len(shapes))]
    cs = [synth.contone(s, h, ww) for s, (h, ww) in zip(seeds, shapes)]
    flat = np.concatenate([c.ravel() for c in cs]).astype(np.float32)
    return w, seeds, cs, flat


@pytest.mark.parametrize("prec", [hb.HS_BF16, hb.HS_FP32])
def test_pages_match_oracle(orc, prec):
    """Pages of different sizes in one call (one fused launch for BF16):
    every page's bits equal the oracle's off the margin."""
    _say("infer pages", prec)
    w, seeds, cs, flat = _pages_inputs(PAGES, 41)
    bits, lg, st = hb.halftone_infer_pages(to_dev(w), to_dev(flat), seeds_t(seeds), PAGES,
                                           precision=prec, recheck_tau=0.055, logits=True,
                                           stats=True)
    bits, lg, st = bits.cpu().numpy(), lg.cpu().numpy(), st.cpu().numpy()
    off = 0
    nnear = 0
    for (h, ww), s, c in zip(PAGES, seeds, cs):
        ref = _oracle_logits(orc, w, c[None], [s], 0)[0]
        b = bits[off:off + h * ww].reshape(h, ww)
        l = lg[off:off + h * ww].reshape(h, ww)
        m = parity_mask(orc, ref)
        assert np.array_equal(b[m], (ref >= 0)[m].astype(np.uint8)), (h, ww)
        if prec == hb.HS_BF16:
            near = np.abs(l) < 0.055
            nnear += int(near.sum())
            assert np.abs(l[near] - ref[near]).max(initial=0.0) <= 0.055 / 8, (h, ww)
            near16 = np.abs(l) < 0.055 / 4
            assert np.abs(l[near16] - ref[near16]).max(initial=0.0) <= 5e-4, (h, ww)
            assert np.abs(l - ref).max() < 0.055
        else:
            assert np.abs(l - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())
        off += h * ww
    if prec == hb.HS_BF16:
        assert st[0] >= nnear > 0


def test_pages_of_one_size_equal_the_batch_call(orc):
    """B equal pages through the pages entry point give exactly the bits and
    logits of the uniform batch call (same kernels, same page table)."""
    B, H, W = 3, 70, 150
    seeds = [61, 62, 63]
    w, c = inputs(seeds, H, W)
    b1, l1 = hb.halftone_infer(to_dev(w), to_dev(c), seeds_t(seeds), 0, hb.HS_BF16, 0.055,
                               logits=True)
    b2, l2 = hb.halftone_infer_pages(to_dev(w), to_dev(c.ravel()), seeds_t(seeds),
                                     [(H, W)] * B, precision=hb.HS_BF16, recheck_tau=0.055,
                                     logits=True)
    assert torch.equal(b1.reshape(-1), b2) and torch.equal(l1.reshape(-1), l2)


def test_c5_pages_full_size_sampled(orc):
    """The uneven-batch workload at its full size: 48 pages of 600..4960 x
    800..7016 (about 0.5 Gpx) in one call; the oracle is evaluated one
    receptive field at a time on sampled pixels of every page (corners,
    centre, random points)."""
    shapes = synth.page_sizes(3_000_000)
    seeds = [3_000_000 + i for i in range(len(shapes))]
    dev = device()
    _say("infer C5 pages", sum(h * w for h, w in shapes))
    flat = torch.cat([synth.contone_torch(s, h, w, dev).reshape(-1)
                      for s, (h, w) in zip(seeds, shapes)])
    w = synth.he_weights(42)
    bits, lg, st = hb.halftone_infer_pages(to_dev(w), flat, seeds_t(seeds), shapes,
                                           precision=hb.HS_BF16, recheck_tau=0.055,
                                           logits=True, stats=True)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[0] > 0 and 0 <= st[2] <= st[0]
    rng = np.random.default_rng(5)
    wd = w.astype(np.float64)
    off = 0
    for (h, ww), s in zip(shapes, seeds):
        pts = [(0, 0), (0, ww - 1), (h - 1, 0), (h - 1, ww - 1), (h // 2, ww // 2)]
        pts += [tuple(int(v) for v in p) for p in rng.integers(0, [h, ww], size=(4, 2))]
        for (y, x) in pts:
            y0, y1, x0, x1 = max(0, y - 6), min(h, y + 7), max(0, x - 6), min(ww, x + 7)
            rows = [flat[off + yy * ww + x0: off + yy * ww + x1] for yy in range(y0, y1)]
            cimg = torch.stack(rows).cpu().numpy()
            zc = np.array([[orc.normal(s, yy * ww + xx, 1, 0) for xx in range(x0, x1)]
                           for yy in range(y0, y1)])
            ref = float(orc.policy_forward_window(wd, cimg.astype(np.float64), zc, y - y0,
                                                  y - y0 + 1, x - x0, x - x0 + 1)[0, 0])
            o = off + y * ww + x
            if abs(orc.sigmoid(ref) - 0.5) > P_MARGIN:
                assert int(bits[o]) == int(ref >= 0), ((h, ww), y, x, ref)
            lo = float(lg[o])
            band = 5e-4 if abs(lo) < 0.055 / 4 else 0.055 / 8 if abs(lo) < 0.055 else 0.055
            assert abs(lo - ref) < band, ((h, ww), y, x)
        off += h * ww
