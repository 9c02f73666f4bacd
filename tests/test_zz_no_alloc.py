"""GPU test of halftone_infer_noalloc, the inference call for callers that
cannot allocate: through the C ABI it must give exactly what halftone_infer
gives with a caller workspace (bits, logits and statistics), on two calls in
a row of which the second is smaller (the static scratch keeps the first
call's contents), in every precision, and it must refuse an input whose
workspace exceeds the scratch before any device work."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import inputs, seeds_t, to_dev
from paper_2304_12152_amd import binding as hb

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(prec, seeds, H, W, tau=None):
    w, c = inputs(seeds, H, W)
    wt, ct, st = to_dev(w), to_dev(c), seeds_t(seeds)
    ref = hb.halftone_infer(wt, ct, st, precision=prec, recheck_tau=tau, logits=True, stats=True)
    got = hb.halftone_infer_noalloc(wt, ct, st, precision=prec, recheck_tau=tau, logits=True,
                                    stats=True)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("prec", [hb.HS_BF16, hb.HS_FP16, hb.HS_FP32])
def test_noalloc_equals_the_workspace_call_twice(prec):
    # first call the larger input, then a smaller one with other seeds
    big = (3, 256, 300) if prec != hb.HS_FP32 else (2, 200, 220)
    small = (1, 37, 91)
    for shape, seed0 in ((big, 11), (small, 101)):
        B, H, W = shape
        _say("noalloc", prec, shape)
        ref, got = _both(prec, list(range(seed0, seed0 + B)), H, W)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (prec, shape)
        assert got[2][0].item() > 0 or prec == hb.HS_FP32


def test_noalloc_wide_band_fills_the_lists():
    # every pixel through both recheck stages: the largest use of the lists
    _say("noalloc wide band")
    ref, got = _both(hb.HS_BF16, [7, 8], 120, 140, tau=1e30)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    assert got[2][0].item() == 2 * 120 * 140


def test_noalloc_refuses_inputs_beyond_the_scratch():
    lib = hb.lib()
    limit = 64 << 20
    assert lib.halftone_infer_workspace_size(3, 1024, 1024, hb.HS_BF16) <= limit
    assert lib.halftone_infer_workspace_size(8, 1024, 1024, hb.HS_BF16) > limit
    w, c = inputs([1], 16, 16)
    wt, st = to_dev(w), seeds_t([1] * 8)
    ct = torch.zeros((8, 1024, 1024), dtype=torch.float32, device=wt.device)
    with pytest.raises(hb.HalftoneError) as e:
        hb.halftone_infer_noalloc(wt, ct, st)
    assert e.value.code == hb.HS_EWORKSPACE
    ct = torch.zeros((1, 600, 600), dtype=torch.float32, device=wt.device)
    with pytest.raises(hb.HalftoneError) as e:
        hb.halftone_infer_noalloc(wt, ct, st[:1], precision=hb.HS_FP32)
    assert e.value.code == hb.HS_EWORKSPACE
