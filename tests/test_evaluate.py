"""The blue-noise evaluation: the ring populations it weights the spectrum
with agree with the oracle's ring rule (host), and one small run on the GPU."""
import numpy as np
import pytest

from paper_2304_12152_amd import evaluate


@pytest.mark.parametrize("P", [32, 64])
def test_ring_counts_follow_the_ring_rule(orc, P):
    ref = np.zeros(orc.ring_index(P // 2, P // 2, P) + 1, dtype=int)
    for u in range(P):
        for v in range(P):
            ref[orc.ring_index(u, v, P)] += 1
    np.testing.assert_array_equal(evaluate._ring_counts(P), ref)
    assert ref.sum() == P * P


@pytest.mark.gpu
def test_bluenoise_summary_on_the_gpu():
    """The evaluation end to end on one small page per gray: Floyd-Steinberg
    keeps the tone, every ring is reported, and the policy runs in the
    planner's precision with its calibrated band (at least the default)."""
    from paper_2304_12152_amd import binding as hb
    from paper_2304_12152_amd import evaluate, synth
    res = evaluate.bluenoise(synth.he_weights(42), grays=(80,), B=2, H=128, W=128, P=32)
    rec = res["80"]
    assert abs(rec["fs"]["fill"] - 80 / 255) < 0.01
    assert len(rec["policy"]["rapsd_db"]) == 16 and len(rec["fs"]["anis_db"]) == 16
    assert res["precision"] == "fp16"  # the planner's choice for the He policy
    assert rec["policy"]["bands"]["tau"] >= hb.RECHECK_TAU[hb.HS_FP16]
    assert 0.0 <= rec["policy"]["fill"] <= 1.0
    assert abs(sum(rec["policy"]["logit_hist"]) - 1.0) < 1e-5
