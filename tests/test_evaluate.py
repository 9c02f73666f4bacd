"""Host logic of the blue-noise evaluation: the ring populations it weights
the spectrum with agree with the oracle's ring rule."""
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
