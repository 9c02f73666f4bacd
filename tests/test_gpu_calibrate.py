"""The recheck band must exceed the 16-bit pass's logit error, which depends
on the weights. A policy whose layer-6 weights are 20 times the He policy's
has 20 times its logits and logit error, beyond the default band;
`calibrate.recheck_tau` measures the band for it, and with that band the
BF16 and FP16 bits equal the FP32 path's off the margin on other images."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import device, inputs, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import calibrate

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _loud_head(w, s=20.0):
    w = w.copy()
    w[-(32 * 9 + 1):] *= s  # layer 6: W6[1][32][3][3] and its bias
    return w


@pytest.mark.parametrize("prec", [hb.HS_BF16, hb.HS_FP16])
def test_calibrated_band_keeps_the_bits(prec):
    _say("calibrated recheck band", prec)
    w, _ = inputs([0], 1, 1)
    wt = to_dev(_loud_head(w))
    seeds = [31, 32]
    c = inputs(seeds, 192, 256)[1]
    ct, st = to_dev(c), seeds_t(seeds)
    err = calibrate.max_logit_error(wt, prec, ct, st)
    assert err > hb.RECHECK_TAU[prec], err  # the default band would not hold
    tau = calibrate.recheck_tau(wt, prec)  # measured on other images
    assert tau >= calibrate.MARGIN[prec] * 0.5 * err
    seeds2 = [41, 42]
    c2 = inputs(seeds2, 200, 260)[1]
    ct2, st2 = to_dev(c2), seeds_t(seeds2)
    b32, l32 = hb.halftone_infer(wt, ct2, st2, 0, hb.HS_FP32, logits=True)
    b16, l16 = hb.halftone_infer(wt, ct2, st2, 0, prec, tau, logits=True)
    off = l32.abs() > 4.1e-4
    assert int(((b16 != b32) & off).sum()) == 0
    assert float((l16 - l32).abs().max()) < tau


def test_calibration_argument_errors():
    w, _ = inputs([0], 1, 1)
    with pytest.raises(ValueError):
        calibrate.recheck_tau(to_dev(w), hb.HS_FP32)
    with pytest.raises(ValueError):
        calibrate.recheck_tau(to_dev(w), hb.HS_BF16,
                              contone=torch.zeros((1, 8, 8), device=device()))


def test_plan_prices_the_options():
    """For the He policy both 16-bit passes list well under the ~4% at which
    the FP32 path would be cheaper; FP16 lists fewer and wins."""
    _say("calibration plan")
    w, _ = inputs([0], 1, 1)
    p = calibrate.plan(to_dev(w))
    o = p["options"]
    assert set(o) == {hb.HS_FP32, hb.HS_BF16, hb.HS_FP16}
    assert 0.0 < o[hb.HS_FP16]["listed"] < o[hb.HS_BF16]["listed"] < 0.02
    assert p["precision"] == hb.HS_FP16
    assert p["bands"]["tau"] == o[hb.HS_FP16]["bands"]["tau"] >= hb.RECHECK_TAU[hb.HS_FP16]
    assert o[hb.HS_FP32]["ns_per_px"] > o[hb.HS_BF16]["ns_per_px"]
    # the BF16 bands: the FP16 cone stage's between the pass's and the split's
    bb = o[hb.HS_BF16]["bands"]
    assert bb["tau"] > bb["tau16"] > bb["tau2"] >= 1.5e-4
    e = bb["errors"]
    assert e["pass"] > e["cone16"] > e["split"] > 0.0 and not e["overflow"]
