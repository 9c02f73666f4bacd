"""Helpers of the GPU parity tests: device fixtures and oracle references."""
import numpy as np
import torch

from paper_2304_12152_amd import binding as hb
from paper_2304_12152_amd import synth

# The bit decision of the paper's test phase is compared wherever the FP32
# margin |p - 0.5| exceeds 1e-4 (|x| > 2 atanh(2e-4) ~ 4.0e-4).
P_MARGIN = 1e-4


def device():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def seeds_t(seeds):
    return to_dev(np.asarray(seeds, dtype=np.int64))


def parity_mask(orc, logits64):
    return np.abs(orc.sigmoid(logits64) - 0.5) > P_MARGIN


def inputs(seeds, H, W, wseed=42):
    w = synth.he_weights(wseed)
    c = synth.contone_batch(seeds, H, W)
    return w, c


def oracle_threads():
    """Threads for the oracle's conv loops in the large parity cases (the
    results are bit-identical for any count): the host's cores, at most 16."""
    import os
    return max(1, min(16, os.cpu_count() or 1))
