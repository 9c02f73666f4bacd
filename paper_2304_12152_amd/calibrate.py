"""Recheck bands of the 16-bit inference paths for a given weight set.

The exact-bit scheme of the TEST procedure (Algorithm 1) recomputes every
pixel whose 16-bit logit lies within recheck_tau of the threshold (of the
nearest level threshold for multitoning), then decides each such pixel in
the first recheck stage whose own error is below that stage's band:
  tau    the fused BF16 (or FP16) pass's band;
  tau16  the FP16 cone stage's (after a BF16 pass only);
  tau2   the split-BF16 cone stage's; the rest go to the FP32 stage.
Every band must exceed its stage's largest logit error, and those errors
depend on the weights: for the He-initialised policy the BF16 pass errs by
at most 0.042 and the FP16 pass by 0.0050 on 8 x 1024 x 1024 synthetic
contones, while a trained policy with large activations and cancelling terms
reached 4.5 and 0.83 on the same images. `bands` measures all three stages
with the library's own calls -- the FP32 path against the fused pass with no
recheck, and against a packed policy's call that lists every pixel and lets
one stage decide all of them -- and returns a margin times each largest
error, never less than the He-policy defaults. They are empirical bounds on
the calibration data, not proofs; the contones default to the synthetic
recipe of `synth.contone`.

    b = calibrate.bands(weights, hb.HS_BF16)
    pol = hb.Policy(weights)
    bits = hb.halftone_policy_infer(pol, contone, seeds, precision=hb.HS_BF16,
                                    recheck_tau=b["tau"], recheck_tau16=b["tau16"],
                                    recheck_tau2=b["tau2"])

`plan` also prices the options: with a band wide enough to list a few
percent of the pixels, the FP32 path becomes the cheaper exact one.

The FP8 pass (HS_FP8) also needs activation scales: `fp8_policy` measures
the largest activation of layers 1..4 in the FP32 forward on the
calibration batch (`halftone_layer_max`) and makes a packed policy's FP8
copy from them; `bands(weights, hb.HS_FP8)` does so when it is given no
such policy and returns it under "policy", since the band holds for those
scales only.
"""
import numpy as np

from . import binding as hb
from . import synth

MARGIN = {hb.HS_BF16: 1.3, hb.HS_FP16: 1.5, hb.HS_FP8: 1.5}
CONE_MARGIN = 2.0     # the cone stages' bands over their largest measured error
TAU2_FLOOR = 1.5e-4   # the split stage's band is never below this (the library's floor)

# Costs per pixel measured on one MI355X for 8 x 1024 x 1024 (ns): the fused
# 16-bit pass (BF16 0.565 ms, FP16 0.570 ms per batch), one listed pixel in
# the FP16 cone stage and in the split stage (0.332 ms for 25,094), and the
# FP32 per-layer path (1,389 Mpx/s).
COST_FUSED_NS = {hb.HS_BF16: 0.067, hb.HS_FP16: 0.068}
COST_CONE16_NS = 6.0
COST_SPLIT_NS = 13.2
COST_FP32_NS = 0.720


def _batch(weights, contone, seeds, who):
    import torch
    dev = weights.device
    if contone is None:
        seeds = [101, 102] if seeds is None else list(seeds)
        contone = torch.tensor(synth.contone_batch(seeds, 512, 512), device=dev)
    if seeds is None:
        raise ValueError(who + ": seeds are needed with a caller's contone batch")
    st = torch.as_tensor(np.asarray(seeds, dtype=np.int64)).to(dev)
    return contone, st


def _pages(contone, levels):
    B, H, W = contone.shape
    return contone.reshape(-1), [(H, W)] * B


def _thresholds(levels):
    j = np.arange(levels - 1, dtype=np.float64)
    return np.log((2.0 * j + 1.0) / (2.0 * levels - 3.0 - 2.0 * j))


def _distance(x, levels):
    """|x - nearest level threshold| (|x| for binary output)."""
    import torch
    if levels == 2:
        return x.abs()
    thr = torch.as_tensor(_thresholds(levels), dtype=x.dtype, device=x.device)
    return (x.reshape(-1, 1) - thr).abs().min(dim=1).values.reshape(x.shape)


def fp8_policy(weights, contone=None, seeds=None, policy=None):
    """A packed Policy of `weights` (or `policy`, packed from them) with its
    FP8 copy, scaled for the largest activations of layers 1..4 in the FP32
    forward over the calibration batch (default: 2 synthetic 512 x 512
    contones, seeds 101 and 102)."""
    contone, st = _batch(weights, contone, seeds, "fp8_policy")
    mx = hb.halftone_layer_max(weights, contone, st).cpu().numpy()
    pol = hb.Policy(weights) if policy is None else policy
    return pol.set_fp8(mx[:4])


def stage_errors(weights, precision, contone, seeds, levels=2, policy=None):
    """Largest |x - x_32| of each stage over the batch (device tensors:
    weights FP32, contone [B, H, W] FP32, seeds int64): "pass" the fused
    pass (the BF16 re-run if an FP16 pass overflowed or an FP8 pass
    saturated, then "overflow" is True), "cone16" the FP16 cone stage (BF16
    only; cones it passes on for overflow are not counted) and "split" the
    split stage. HS_FP8 runs on `policy`, which must have its FP8 copy."""
    flat, shapes = _pages(contone, levels)
    _, l32 = hb.halftone_infer_pages(weights, flat, seeds, shapes, precision=hb.HS_FP32,
                                     logits=True, levels=levels)
    pol = hb.Policy(weights) if policy is None else policy
    if precision == hb.HS_FP8:
        _, l16, st = hb.halftone_policy_infer(pol, flat, seeds, shapes, precision=precision,
                                              recheck_tau=0.0, logits=True, stats=True,
                                              levels=levels)
    else:
        _, l16, st = hb.halftone_infer_pages(weights, flat, seeds, shapes, precision=precision,
                                             recheck_tau=0.0, logits=True, stats=True,
                                             levels=levels)
    out = {"overflow": int(st[3]) != 0}
    if out["overflow"]:
        _, l16 = hb.halftone_infer_pages(weights, flat, seeds, shapes, precision=hb.HS_BF16,
                                         recheck_tau=0.0, logits=True, levels=levels)
    out["pass"] = float((l16 - l32).abs().max())
    # every pixel listed; one stage decides all of them (tau2 = 0: none go
    # on to FP32; tau16 = 1e-30: the FP16 stage decides all but overflowed
    # cones and exact zeros, which the split stage decides)
    for name, t16 in (("cone16", 1e-30), ("split", 0.0)):
        if name == "cone16" and precision != hb.HS_BF16:
            continue
        _, lc = hb.halftone_policy_infer(pol, flat, seeds, shapes, precision=hb.HS_BF16,
                                         recheck_tau=1e30, recheck_tau16=t16, recheck_tau2=0.0,
                                         logits=True, levels=levels)
        out[name] = float((lc - l32).abs().max())
    return out


def max_logit_error(weights, precision, contone, seeds):
    """Largest |x_16 - x_32| of the fused 16-bit pass over the batch."""
    _, l32 = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, hb.HS_FP32,
                               logits=True)
    _, l16, st = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, precision, 0.0,
                                   logits=True, stats=True)
    if int(st[3]) != 0:
        _, l16 = hb.halftone_infer(weights, contone, seeds, hb.HS_NOISE_GAUSS, hb.HS_BF16, 0.0,
                                   logits=True)
    return float((l16 - l32).abs().max())


def bands(weights, precision=hb.HS_BF16, contone=None, seeds=None, margin=None, levels=2,
          policy=None):
    """The three bands for `weights` (a device tensor) from the stage errors
    on the calibration batch (default: 2 synthetic 512 x 512 contones, seeds
    101 and 102): {"tau", "tau16", "tau2", "errors"}; tau16 is 0 (no FP16
    cone stage) after an FP16 or FP8 pass. HS_FP8: on `policy` if it has
    its FP8 copy, else on one made by fp8_policy from the calibration batch
    (returned under "policy"); tau is at least 8 times the BF16 default,
    so that the BF16 re-run after a saturation (tau / 8) keeps that band."""
    if precision not in MARGIN:
        raise ValueError("bands: precision must be HS_BF16, HS_FP16 or HS_FP8")
    contone, st = _batch(weights, contone, seeds, "bands")
    if precision == hb.HS_FP8 and (policy is None or policy.act_max is None):
        policy = fp8_policy(weights, contone, st.tolist(), policy)
    e = stage_errors(weights, precision, contone, st, levels, policy)
    m = MARGIN[precision] if margin is None else margin
    if precision == hb.HS_FP8:
        tau = max(m * e["pass"], 8.0 * hb.RECHECK_TAU[hb.HS_BF16])
    else:
        tau = max(m * e["pass"], hb.RECHECK_TAU[precision])
        if e["overflow"]:
            tau = max(tau, 8.0 * hb.RECHECK_TAU[precision])
    tau2 = max(CONE_MARGIN * e["split"], TAU2_FLOOR)
    tau16 = max(CONE_MARGIN * e["cone16"], 2.0 * tau2) if "cone16" in e else 0.0
    out = {"tau": tau, "tau16": tau16, "tau2": tau2, "errors": e}
    if precision == hb.HS_FP8:
        out["policy"] = policy
    return out


def recheck_tau(weights, precision=hb.HS_BF16, contone=None, seeds=None, margin=None):
    """recheck_tau for `weights` (a device tensor): margin x the largest
    logit error of the fused pass on the calibration batch (default: 2
    synthetic 512 x 512 contones, seeds 101 and 102), at least
    RECHECK_TAU[precision]."""
    if precision not in (hb.HS_BF16, hb.HS_FP16):
        raise ValueError("recheck_tau: precision must be HS_BF16 or HS_FP16 (bands for HS_FP8)")
    contone, st = _batch(weights, contone, seeds, "recheck_tau")
    err = max_logit_error(weights, precision, contone, st)
    m = MARGIN[precision] if margin is None else margin
    return max(m * err, hb.RECHECK_TAU[precision])


def plan(weights, contone=None, seeds=None, levels=2):
    """The cheapest exact-bit precision for `weights` with `levels` output
    levels: for BF16 and FP16 the calibrated bands and the shares of the
    calibration batch's pixels inside them (distance to the nearest level
    threshold), priced with the measured per-pixel costs against the FP32
    path. An FP16 pass that overflows costs both fused passes and lists
    within 8 tau. Returns {"precision", "bands", "options"}."""
    contone, st = _batch(weights, contone, seeds, "plan")
    flat, shapes = _pages(contone, levels)
    opts = {hb.HS_FP32: {"bands": None, "listed": 0.0, "ns_per_px": COST_FP32_NS}}
    for prec in (hb.HS_BF16, hb.HS_FP16):
        b = bands(weights, prec, contone, st.tolist(), levels=levels)
        over = b["errors"]["overflow"]
        _, x = hb.halftone_infer_pages(weights, flat, st, shapes,
                                       precision=hb.HS_BF16 if over else prec, recheck_tau=0.0,
                                       logits=True, levels=levels)
        d = _distance(x, levels)
        tau = 8.0 * b["tau"] if (over and prec == hb.HS_FP16) else b["tau"]
        listed = float((d < tau).double().mean())
        fused = COST_FUSED_NS[prec] + (COST_FUSED_NS[hb.HS_BF16] if over else 0.0)
        if prec == hb.HS_BF16:
            to_split = float((d < b["tau16"]).double().mean())
            ns = fused + listed * COST_CONE16_NS + to_split * COST_SPLIT_NS
        else:
            ns = fused + listed * COST_SPLIT_NS
        opts[prec] = {"bands": b, "listed": listed, "ns_per_px": ns}
    best = min(opts, key=lambda p: opts[p]["ns_per_px"])
    return {"precision": best, "bands": opts[best]["bands"], "options": opts}
