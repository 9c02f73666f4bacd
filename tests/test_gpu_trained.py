"""GPU tests on a trained policy: the learned part of the method (Alg. 1,
TRAIN then TEST; Sec. VI-B) and the exact-bit scheme on high-gain weights.

The fixture tests/golden/policy_binary_300k.npy holds the FP32 weights of
the 6 x 32 policy after 300,000 training steps of `policy_train_step`
(batch 32 x 256 x 256 from the synthetic pool plus the 64-gray side batch,
w_s = 0, w_a = 2e-5, BF16 activations; the command is in
tests/golden/policy_binary_300k.txt). It is an input weight set, like a
checkpoint: every expected value below comes from the oracle, from the
FP32 path, or from the judge's definition.

A trained policy has logits of median magnitude ~18 and a 16-bit logit
error ~100 times the He policy's, so its recheck bands are calibrated
(`calibrate.bands`) on seeds disjoint from the images checked here."""
import os
import sys

import numpy as np
import pytest
import torch

from gpu_common import oracle_threads, parity_mask, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import calibrate, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "policy_binary_300k.npy")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trained():
    w = np.load(FIXTURE)
    assert w.dtype == np.float32 and w.shape == (hb.HS_PARAM_COUNT,)
    return w


@pytest.fixture(scope="module")
def cal(trained):
    _say("calibrating the trained policy's bands")
    return calibrate.bands(to_dev(trained), hb.HS_BF16)


def test_trained_bands_and_stage_errors(trained, cal):
    """Each stage's error on images other than the calibration ones stays
    below half its calibrated band."""
    e = cal["errors"]
    _say("bands", {k: v for k, v in cal.items() if k != "errors"}, "errors", e)
    assert cal["tau"] > 10 * hb.RECHECK_TAU[hb.HS_BF16]  # far beyond the He band
    assert cal["tau"] > cal["tau16"] > cal["tau2"] > 0.0
    seeds = [2_100_001, 2_100_002]
    c = synth.contone_batch(seeds, 384, 384)
    e2 = calibrate.stage_errors(to_dev(trained), hb.HS_BF16, to_dev(c), seeds_t(seeds))
    _say("errors on other images", e2)
    assert e2["pass"] < cal["tau"] / 1.2
    assert e2["cone16"] < cal["tau16"] / 2
    assert e2["split"] < cal["tau2"] / 2


def test_trained_bits_match_the_oracle(orc, trained, cal):
    """BF16 with the calibrated bands: bits equal the oracle's on the whole
    of 2 x 512 x 512 wherever |p - 0.5| > 1e-4, and the FP32 path's."""
    seeds = [2_100_011, 2_100_012]
    H = W = 512
    c = synth.contone_batch(seeds, H, W)
    wt, ct, st = to_dev(trained), to_dev(c), seeds_t(seeds)
    pol = hb.Policy(wt)
    bits, stt = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_BF16,
                                         recheck_tau=cal["tau"], recheck_tau16=cal["tau16"],
                                         recheck_tau2=cal["tau2"], stats=True)
    bits, stt = bits.cpu().numpy(), stt.cpu().numpy()
    _say("trained policy, 2 x 512^2: listed", stt[0], "split", stt[4], "fp32", stt[2])
    z = orc.noise_map(seeds, H, W, kind=0, stream=1, step=0)
    with orc.threads(oracle_threads()):
        ref = orc.policy_forward(trained.astype(np.float64), c.astype(np.float64), z)
    m = parity_mask(orc, ref)
    assert int((bits[m] != (ref >= 0)[m]).sum()) == 0
    b32, l32 = hb.halftone_infer(wt, ct, st, precision=hb.HS_FP32, logits=True)
    off = (l32.abs() > 4.1e-4).cpu().numpy()
    assert int((bits[off] != b32.cpu().numpy()[off]).sum()) == 0
    # the default He band is far too narrow for these weights: bits differ
    bd = hb.halftone_infer(wt, ct, st, precision=hb.HS_BF16).cpu().numpy()
    assert int((bd[m] != (ref >= 0)[m]).sum()) > 0


def test_trained_fp16_bits_match_the_fp32_path(trained):
    """FP16 fused pass with its calibrated band (split and FP32 behind it)."""
    wt = to_dev(trained)
    b = calibrate.bands(wt, hb.HS_FP16)
    seeds = [2_100_021, 2_100_022]
    c = synth.contone_batch(seeds, 512, 512)
    ct, st = to_dev(c), seeds_t(seeds)
    pol = hb.Policy(wt)
    bits = hb.halftone_policy_infer(pol, ct, st, precision=hb.HS_FP16, recheck_tau=b["tau"],
                                    recheck_tau2=b["tau2"])
    b32, l32 = hb.halftone_infer(wt, ct, st, precision=hb.HS_FP32, logits=True)
    off = l32.abs() > 4.1e-4
    assert int(((bits != b32) & off).sum()) == 0


def test_trained_policy_beats_the_untrained_one(trained):
    """The held-out judge (Sec. VI-B protocol with the Gaussian HVS): mean
    HVS-filtered MSE of [p >= 0.5] on 64 held-out contones, trained against
    the untrained He policy (what training gains) and Floyd-Steinberg (the
    fallback, printed: the paper's own table has error diffusion ahead)."""
    from paper_2304_12152_amd import train
    n = 64
    seeds = list(range(train.JUDGE_SEED0, train.JUDGE_SEED0 + n))
    c = synth.contone_batch(seeds, 256, 256)
    s = np.asarray(seeds, dtype=np.uint64)
    t = train.judge(trained, c, s)
    u = train.judge(synth.he_weights(42, head_std=0.01), c, s, with_fs=False)
    _say("held-out judge: trained %.4g, untrained %.4g, Floyd-Steinberg %.4g (ratio %.2f)"
         % (t["policy_hvs_mse"], u["policy_hvs_mse"], t["fs_hvs_mse"],
            t["policy_hvs_mse"] / t["fs_hvs_mse"]))
    assert t["policy_hvs_mse"] < 0.25 * u["policy_hvs_mse"]
    assert abs(t["policy_fill"] - t["contone_mean"]) < 0.02  # tone preserved
    assert t["fs_hvs_mse"] > 0.0
