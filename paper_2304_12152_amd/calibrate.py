"""Recheck band of the 16-bit inference passes for a given weight set.

The exact-bit scheme of the TEST procedure (Algorithm 1) recomputes every
pixel whose BF16 (or FP16) logit lies within recheck_tau of the threshold,
so recheck_tau must exceed the largest logit error of the 16-bit pass. That
error depends on the weights: for the He-initialised policy it is 0.042
(BF16) and 0.0050 (FP16) on 8 x 1024 x 1024 synthetic contones, but a
trained policy with large activations and cancelling terms reached 4.5 and
0.83 on the same images. `recheck_tau` measures it on a calibration batch
with the library's own calls (the FP32 path against the 16-bit pass with no
recheck) and returns `margin` times the largest error, never less than the
He-policy default. It is an empirical bound on the calibration data, not a
proof; the contones default to the synthetic recipe of `synth.contone`.

    tau = calibrate.recheck_tau(weights, hb.HS_BF16)
    bits = hb.halftone_infer(weights, contone, seeds, precision=hb.HS_BF16,
                             recheck_tau=tau)

`plan` also prices the options: with a band wide enough to list a few
percent of the pixels, the FP32 path becomes the cheaper exact one.
"""
import numpy as np

from . import binding as hb
from . import synth

MARGIN = {hb.HS_BF16: 1.3, hb.HS_FP16: 1.5}

# Costs per pixel measured on one MI355X for 8 x 1024 x 1024 (ns): the fused
# 16-bit pass (BF16 0.57 ms, FP16 0.59 ms per batch), one listed pixel in the
# split stage (383 us for 25,094 cones), and the FP32 per-layer path (6.06 ms).
COST_FUSED_NS = {hb.HS_BF16: 0.068, hb.HS_FP16: 0.070}
COST_LISTED_NS = 15.3
COST_FP32_NS = 0.722


def _logits(weights, precision, contone, seeds):
    """FP32 logits and the 16-bit pass's unrechecked logits."""
    _, l32 = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, hb.HS_FP32,
                               logits=True)
    _, l16, st = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, precision, 0.0,
                                   logits=True, stats=True)
    if int(st[3]) != 0:
        # the FP16 pass overflowed and the BF16 pass decided: measure that one
        _, l16 = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, hb.HS_BF16, 0.0,
                                   logits=True)
    return l32, l16


def max_logit_error(weights, precision, contone, seeds):
    """Largest |x_16 - x_32| of the 16-bit pass over the batch (device
    tensors: weights FP32, contone [B, H, W] FP32, seeds int64)."""
    l32, l16 = _logits(weights, precision, contone, seeds)
    return float((l16 - l32).abs().max())


def plan(weights, contone=None, seeds=None):
    """The cheapest exact-bit precision for `weights` (binary output): for
    BF16 and FP16 the calibrated band and the share of the calibration
    batch's pixels inside it, priced with the measured per-pixel costs
    against the FP32 path. Returns {"precision", "recheck_tau", "options"}."""
    import torch
    dev = weights.device
    if contone is None:
        seeds = [101, 102] if seeds is None else list(seeds)
        contone = torch.tensor(synth.contone_batch(seeds, 512, 512), device=dev)
    if seeds is None:
        raise ValueError("plan: seeds are needed with a caller's contone batch")
    st = torch.as_tensor(np.asarray(seeds, dtype=np.int64)).to(dev)
    opts = {hb.HS_FP32: {"recheck_tau": 0.0, "listed": 0.0, "ns_per_px": COST_FP32_NS}}
    for prec in (hb.HS_BF16, hb.HS_FP16):
        l32, l16 = _logits(weights, prec, contone, st)
        tau = max(MARGIN[prec] * float((l16 - l32).abs().max()), hb.RECHECK_TAU[prec])
        listed = float((l16.abs() < tau).double().mean())
        opts[prec] = {"recheck_tau": tau, "listed": listed,
                      "ns_per_px": COST_FUSED_NS[prec] + listed * COST_LISTED_NS}
    best = min(opts, key=lambda p: opts[p]["ns_per_px"])
    return {"precision": best, "recheck_tau": opts[best]["recheck_tau"], "options": opts}


def recheck_tau(weights, precision=hb.HS_BF16, contone=None, seeds=None, margin=None):
    """recheck_tau for `weights` (a device tensor): margin x the largest
    logit error on the calibration batch (default: 2 synthetic 512 x 512
    contones, seeds 101 and 102), at least RECHECK_TAU[precision]."""
    import torch
    if precision not in MARGIN:
        raise ValueError("recheck_tau: precision must be HS_BF16 or HS_FP16")
    dev = weights.device
    if contone is None:
        seeds = [101, 102] if seeds is None else list(seeds)
        contone = torch.tensor(synth.contone_batch(seeds, 512, 512), device=dev)
    if seeds is None:
        raise ValueError("recheck_tau: seeds are needed with a caller's contone batch")
    st = torch.as_tensor(np.asarray(seeds, dtype=np.int64)).to(dev)
    err = max_logit_error(weights, precision, contone, st)
    m = MARGIN[precision] if margin is None else margin
    return max(m * err, hb.RECHECK_TAU[precision])
