"""Pins of the COMA estimator (Sec. III-A, Eqs. reinforce, baseline, coma).

The oracle forms R(h) - b_a from the toggle difference dR_a. These tests
check it against the definition evaluated literally (every reward
recomputed from scratch, the score function by finite differences), against
its relation to the Local Expectation estimator, and for unbiasedness by
exhaustive enumeration of every halftone of a small image."""
import itertools

import numpy as np

PRM_SMALL = dict(hvs_r=1, ssim_r=1, hvs_sigma=1.0, ssim_sigma=1.0, w_s=1.0, estimator=1)


def test_coma_equals_literal_definition(orc):
    # b_a = sum_{h'} pi_a(h') R({h', h_-a}), each R evaluated from scratch;
    # d/dx log pi_a(h_a) by a central difference of log(sigmoid) in x
    rng = np.random.default_rng(3)
    B, H, W = 2, 7, 8
    c = rng.uniform(0.05, 0.95, size=(B, H, W))
    x = rng.normal(0.0, 1.5, size=(B, H, W))
    p = 1.0 / (1.0 + np.exp(-x))
    h = (rng.uniform(size=(B, H, W)) < p).astype(np.float64)
    g = orc.coma_grad_logits(h, c, p, PRM_SMALL)
    prm = dict(PRM_SMALL)
    for b in range(B):
        R = orc.reward(h[b:b + 1], c[b:b + 1], prm)[0, 2]
        for (y, xx) in [(0, 0), (3, 4), (6, 7), (2, 1), (5, 6)]:
            t1 = h[b:b + 1].copy(); t1[0, y, xx] = 1.0
            t0 = h[b:b + 1].copy(); t0[0, y, xx] = 0.0
            R1 = orc.reward(t1, c[b:b + 1], prm)[0, 2]
            R0 = orc.reward(t0, c[b:b + 1], prm)[0, 2]
            pa = p[b, y, xx]
            base = pa * R1 + (1.0 - pa) * R0

            def logpi(xv):
                pv = 1.0 / (1.0 + np.exp(-xv))
                return np.log(pv if h[b, y, xx] == 1.0 else 1.0 - pv)

            e = 1e-5
            score = (logpi(x[b, y, xx] + e) - logpi(x[b, y, xx] - e)) / (2 * e)
            want = -score * (R - base) / B
            assert abs(g[b, y, xx] - want) <= 1e-8 * max(abs(want), 1e-6)


def test_coma_expectation_over_own_action_is_le(orc):
    # given h_-a, E_{h_a ~ pi_a}[g_COMA] = -dR_a p_a (1 - p_a) / B (the Local
    # Expectation gradient in logit space): dR_a does not depend on h_a
    rng = np.random.default_rng(4)
    c = rng.uniform(size=(1, 9, 9))
    p = rng.uniform(0.05, 0.95, size=(1, 9, 9))
    h = (rng.uniform(size=c.shape) < 0.5).astype(np.float64)
    prm = dict(PRM_SMALL)
    le = orc.le_grad_probs(h, c, prm) * p * (1 - p)
    for (y, x) in [(4, 4), (0, 8), (8, 0)]:
        h1 = h.copy(); h1[0, y, x] = 1.0
        h0 = h.copy(); h0[0, y, x] = 0.0
        g1 = orc.coma_grad_logits(h1, c, p, prm)[0, y, x]
        g0 = orc.coma_grad_logits(h0, c, p, prm)[0, y, x]
        pa = p[0, y, x]
        assert abs(pa * g1 + (1 - pa) * g0 - le[0, y, x]) < 1e-15


def test_coma_estimator_is_unbiased_by_enumeration(orc):
    # 3x4 image, radius-1 windows: E_{h~pi}[g_COMA(h)] over all 2^12 halftones
    # equals -dE_pi[R]/dx (E_pi[R] is multilinear in p; central differences
    # in p times dp/dx are exact up to rounding)
    rng = np.random.default_rng(5)
    Hh, Ww = 3, 4
    n = Hh * Ww
    c = rng.uniform(0.1, 0.9, size=(Hh, Ww))
    x = rng.normal(0.0, 1.0, size=n)
    p = 1.0 / (1.0 + np.exp(-x))
    Hs = np.array(list(itertools.product([0.0, 1.0], repeat=n)))
    hs = Hs.reshape(-1, Hh, Ww)
    cs = np.broadcast_to(c, hs.shape).copy()
    prm = dict(PRM_SMALL)
    R = orc.reward(hs, cs, prm)[:, 2]
    ps = np.broadcast_to(p.reshape(Hh, Ww), hs.shape).copy()
    # the oracle averages over its batch; undo the 1/B to get per-sample g
    g = orc.coma_grad_logits(hs, cs, ps, prm).reshape(-1, n) * hs.shape[0]

    def prob(pv):
        return np.prod(np.where(Hs == 1.0, pv, 1.0 - pv), axis=1)

    lhs = prob(p) @ g
    eps = 1e-3
    for a in range(n):
        pp = p.copy(); pp[a] += eps
        pm = p.copy(); pm[a] -= eps
        dEdp = (prob(pp) @ R - prob(pm) @ R) / (2 * eps)
        rhs = -dEdp * p[a] * (1 - p[a])
        assert abs(lhs[a] - rhs) < 1e-11 * max(1.0, abs(rhs)) + 1e-13


def test_coma_zero_when_policy_is_deterministic(orc):
    # p = h exactly (a deterministic policy that took its only action):
    # R(h) = b_a, so the estimator vanishes
    rng = np.random.default_rng(6)
    c = rng.uniform(size=(1, 8, 8))
    h = (rng.uniform(size=c.shape) < 0.5).astype(np.float64)
    g = orc.coma_grad_logits(h, c, h.copy(), PRM_SMALL)
    assert np.abs(g).max() == 0.0
