"""Pins of the optimiser, of Floyd-Steinberg, and of one TRAIN iteration of
Algorithm 1 against torch autograd (float64) with torch.fft and
torch.optim.Adam as the library routines."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2304_12152_amd import synth
from test_oracle_policy import torch_forward, torch_policy


def test_lr_schedule_closed_form(orc):
    assert abs(orc.lr_cosine(0, 1000) - 3e-4) < 1e-18
    assert abs(orc.lr_cosine(1000, 1000) - 1e-5) < 1e-18
    assert abs(orc.lr_cosine(500, 1000) - (3e-4 + 1e-5) / 2) < 1e-18
    assert abs(orc.lr_cosine(250, 1000) - (1e-5 + 0.5 * 2.9e-4 * (1 + math.cos(math.pi / 4)))) < 1e-18


def test_adam_first_step_moves_by_lr(orc):
    rng = np.random.default_rng(0)
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    g = rng.normal(size=50)
    th0 = th.copy()
    orc.adam_step(th, m, v, g, 1, 1e-3)
    np.testing.assert_allclose(np.abs(th - th0), 1e-3 * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(1)
    th = rng.normal(size=40)
    m = np.zeros(40)
    v = np.zeros(40)
    tt = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=40)
        orc.adam_step(th, m, v, g, t, 2e-3)
        tt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_fs_half_gray_is_checkerboard(orc):
    h = orc.floyd_steinberg(np.full((1, 6, 6), 0.5))[0]
    yy, xx = np.mgrid[0:6, 0:6]
    assert np.array_equal(h, ((yy + xx + 1) % 2).astype(np.uint8))


def test_fs_hand_worked(orc):
    # c = [[.3, .6], [.8, .1]] worked by hand: (0,0) 0.3 -> 0 (err .3);
    # (0,1) .6 + .13125 -> 1; (1,0) .8 + .09375 - .05039 -> 1;
    # (1,1) .1 + .01875 - .08398 - .06853 -> 0
    h = orc.floyd_steinberg(np.array([[[0.3, 0.6], [0.8, 0.1]]]))[0]
    assert h.tolist() == [[0, 1], [1, 0]]


def test_fs_tone_preservation(orc):
    c = synth.contone_batch([31, 32], 64, 64).astype(np.float64)
    h = orc.floyd_steinberg(c)
    for b in range(2):
        # error can only leave through the right column and the bottom row
        assert abs(h[b].mean() - c[b].mean()) <= (64 + 64) / (64 * 64)


def _ring_map(P=32):
    return np.array([[int(np.floor(np.hypot(min(u, P - u), min(v, P - v)) + 0.5))
                      for v in range(P)] for u in range(P)])


def _as_loss_torch(pg, P=32):
    B, H, W = pg.shape
    rho = torch.as_tensor(_ring_map(P))
    tot = 0.0
    n = 0
    for b in range(B):
        for ty in range(H // P):
            for tx in range(W // P):
                X = torch.fft.fft2(pg[b, ty * P:(ty + 1) * P, tx * P:(tx + 1) * P])
                ph = (X.real ** 2 + X.imag ** 2) / (P * P)
                for r in range(int(rho.max()) + 1):
                    m = rho == r
                    tot = tot + ((ph[m] - ph[m].mean()) ** 2).sum()
                n += 1
    return tot / n


@pytest.mark.parametrize("noise_kind", [0, 1])
def test_train_step_matches_autograd_and_adam(orc, noise_kind):
    ch = orc.CH
    w0 = synth.he_weights(5, head_std=0.01).astype(np.float64)
    B, H, W = 2, 20, 22
    c = synth.contone_batch([40, 41], H, W).astype(np.float64)
    seeds = np.array([40, 41], dtype=np.uint64)
    cg = synth.gray_batch(2, 32, 64).astype(np.float64)
    gseeds = np.array([900, 901], dtype=np.uint64)
    step, total = 3, 10
    w = w0.copy(); m = np.zeros_like(w); v = np.zeros_like(w)
    out = orc.train_step(w, m, v, c, seeds, cg, gseeds, step, total, noise_kind=noise_kind)
    h = out["actions"].astype(np.float64)
    # the same iteration with torch autograd as the chain rule
    z = orc.noise_map(seeds, H, W, kind=noise_kind, stream=1, step=step)
    zg = orc.noise_map(gseeds, 32, 64, kind=noise_kind, stream=1, step=step)
    s, params = torch_policy(w0, c, z, ch)
    sg, _ = torch_policy(w0, cg, zg, ch)
    for p_ in params:
        p_.requires_grad_(True)
    p = torch.sigmoid(torch_forward(s, params))
    pg = torch.sigmoid(torch_forward(sg, params))
    dR = orc.le_delta(h, c)
    surrogate = (torch.as_tensor(-dR / B) * p).sum()
    loss = surrogate + 0.002 * _as_loss_torch(pg)
    loss.backward()
    want = torch.cat([p_.grad.reshape(-1) for p_ in params]).numpy()
    np.testing.assert_allclose(out["grad"], want, rtol=1e-9, atol=1e-12 * np.abs(want).max())
    # the actions are Bernoulli draws of stream 0 at this step
    u = orc.noise_map(seeds, H, W, kind=1, stream=0, step=step)
    assert np.array_equal(out["actions"], (u < p.detach().numpy()).astype(np.uint8))
    # Adam with the cosine learning rate of this step; the bias corrections
    # use t = step + 1, so torch takes `step` zero-gradient steps first
    # (which leave the parameters and moments untouched)
    lr = orc.lr_cosine(step, total)
    tt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(step):
        tt.grad = torch.zeros_like(tt)
        opt.step()
    tt.grad = torch.tensor(want)
    opt.step()
    np.testing.assert_allclose(w, tt.detach().numpy(), rtol=1e-12, atol=1e-9 * lr)
    met = out["metrics"]
    assert abs(met["lr"] - lr) < 1e-18
    assert abs(met["fill"] - h.mean()) < 1e-15


def test_fs_levels_two_is_binary_fs(orc):
    c = synth.contone_batch([33, 34], 40, 56).astype(np.float64)
    assert np.array_equal(orc.floyd_steinberg_levels(c, 2), orc.floyd_steinberg(c))


def test_fs_levels_exact_levels_carry_no_error(orc):
    # a contone that sits on a level everywhere is reproduced exactly
    for L, k in ((3, 1), (4, 2), (8, 5)):
        c = np.full((1, 9, 13), k / (L - 1.0))
        assert np.all(orc.floyd_steinberg_levels(c, L) == k)


def test_fs_levels_hand_worked(orc):
    # L = 3 (levels 0, 1/2, 1) on [[.3, .9], [.6, .2]] worked by hand:
    # (0,0) .3 -> 1/2, error -.2; (0,1) .9 - .0875 = .8125 -> 1, error
    # -.1875; (1,0) .6 - .0625 - .03516 = .50234 -> 1/2, error .00234;
    # (1,1) .2 - .0125 - .05859 + .00103 = .12993 -> 0
    k = orc.floyd_steinberg_levels(np.array([[[0.3, 0.9], [0.6, 0.2]]]), 3)[0]
    assert k.tolist() == [[1, 2], [1, 0]]


@pytest.mark.parametrize("L", [3, 4])
def test_fs_levels_tone_preservation(orc, L):
    c = synth.contone_batch([35, 36], 64, 64).astype(np.float64)
    k = orc.floyd_steinberg_levels(c, L)
    for b in range(2):
        # the error left at the right column and bottom row is below one
        # level step per pixel there
        assert abs(k[b].mean() / (L - 1) - c[b].mean()) <= (64 + 64) / (64 * 64) / (L - 1)
