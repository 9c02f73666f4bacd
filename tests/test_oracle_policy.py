"""Pins of the oracle's policy network: special cases with a closed form
(delta kernel, bias-only net), the library convolution of PyTorch in float64
for the full stack, and the chain rule checked by autograd and by finite
differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2304_12152_amd import synth


def torch_policy(w, c, z, ch):
    """The stack written with torch's conv2d (zero padding 1), float64."""
    B, H, W = c.shape
    s = torch.stack([torch.as_tensor(c), torch.as_tensor(z)], dim=1).double()
    off = 0
    L = len(ch) - 1
    params = []
    for l in range(L):
        ci, co = ch[l], ch[l + 1]
        Wl = torch.as_tensor(w[off:off + co * ci * 9]).double().reshape(co, ci, 3, 3)
        off += co * ci * 9
        bl = torch.as_tensor(w[off:off + co]).double()
        off += co
        params += [Wl, bl]
    return s, params


def torch_forward(s, params):
    L = len(params) // 2
    x = s
    for l in range(L):
        x = F.conv2d(x, params[2 * l], params[2 * l + 1], padding=1)
        if l < L - 1:
            x = F.relu(x)
    return x[:, 0]


def test_param_count(orc):
    assert orc.param_count() == 37889


def test_delta_kernel_is_identity(orc):
    # one 1->1 layer (with the z channel weighted 0) whose kernel is a centred
    # delta: the output is the contone itself
    ch = (2, 1)
    w = np.zeros(2 * 9 + 1)
    w[4] = 1.0  # W[0][0][1][1]
    rng = np.random.default_rng(1)
    c = rng.uniform(size=(2, 9, 13))
    z = rng.normal(size=(2, 9, 13))
    x = orc.policy_forward(w, c, z, ch=ch)
    assert np.array_equal(x, c)


def test_shifted_delta_kernel_pads_with_zero(orc):
    ch = (2, 1)
    w = np.zeros(19)
    w[0 * 9 + 0 * 3 + 2] = 1.0  # W[0][0][dy=0][dx=2]: reads (y-1, x+1)
    rng = np.random.default_rng(2)
    c = rng.uniform(size=(1, 7, 8))
    x = orc.policy_forward(w, c, np.zeros_like(c), ch=ch)
    want = np.zeros_like(c)
    want[:, 1:, :-1] = c[:, :-1, 1:]
    assert np.array_equal(x, want)


def test_bias_only_net_is_constant(orc):
    ch = (2, 3, 4, 1)
    n = orc.param_count(ch)
    w = np.zeros(n)
    # biases: layer 1 (3 ch) at 2*3*9.., layer 2 (4 ch), layer 3 (1 ch)
    o1 = 3 * 2 * 9
    w[o1:o1 + 3] = [0.5, -1.0, 2.0]
    o2 = o1 + 3 + 4 * 3 * 9
    w[o2:o2 + 4] = [0.25, -0.5, 1.0, 3.0]
    o3 = o2 + 4 + 1 * 4 * 9
    w[o3] = -0.75
    c = np.random.default_rng(3).uniform(size=(1, 6, 5))
    x = orc.policy_forward(w, c, c, ch=ch)
    assert np.all(x == -0.75)


def test_full_stack_matches_torch_conv2d(orc):
    ch = orc.CH
    w = synth.he_weights(42).astype(np.float64)
    c = synth.contone_batch([1, 2], 20, 23).astype(np.float64)
    z = np.random.default_rng(4).normal(size=c.shape)
    x = orc.policy_forward(w, c, z)
    s, params = torch_policy(w, c, z, ch)
    want = torch_forward(s, params).numpy()
    np.testing.assert_allclose(x, want, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("win", [(0, 5, 0, 7), (3, 11, 9, 17), (14, 20, 20, 23), (7, 8, 11, 12)])
def test_window_equals_full(orc, win):
    w = synth.he_weights(7).astype(np.float64)
    c = synth.contone(5, 20, 23).astype(np.float64)
    z = np.random.default_rng(5).normal(size=c.shape)
    full = orc.policy_forward(w, c[None], z[None])[0]
    y0, y1, x0, x1 = win
    part = orc.policy_forward_window(w, c, z, y0, y1, x0, x1)
    np.testing.assert_array_equal(part, full[y0:y1, x0:x1])


def test_threshold_tie_is_white(orc):
    b = orc.threshold(np.array([-1e-300, 0.0, 1e-300, -2.0, 3.0]))
    assert b.tolist() == [0, 1, 1, 0, 1]


def test_backward_matches_torch_autograd(orc):
    ch = orc.CH
    w = synth.he_weights(11).astype(np.float64)
    c = synth.contone_batch([3, 4], 12, 15).astype(np.float64)
    z = np.random.default_rng(6).normal(size=c.shape)
    g = np.random.default_rng(7).normal(size=c.shape)
    gw, gi = orc.policy_backward(w, c, z, g)
    s, params = torch_policy(w, c, z, ch)
    s.requires_grad_(True)
    for p in params:
        p.requires_grad_(True)
    x = torch_forward(s, params)
    (x * torch.as_tensor(g)).sum().backward()
    want = torch.cat([p.grad.reshape(-1) for p in params]).numpy()
    np.testing.assert_allclose(gw, want, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gi, s.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_backward_finite_differences(orc):
    # central differences in FP64 on a small net and image
    ch = (2, 4, 4, 1)
    n = orc.param_count(ch)
    rng = np.random.default_rng(8)
    w = rng.normal(scale=0.5, size=n)
    c = rng.uniform(size=(1, 6, 7))
    z = rng.normal(size=(1, 6, 7))
    g = rng.normal(size=(1, 6, 7))
    gw, _ = orc.policy_backward(w, c, z, g, ch=ch)

    def loss(wv):
        return float((orc.policy_forward(wv, c, z, ch=ch) * g).sum())

    eps = 1e-6
    for i in rng.choice(n, size=25, replace=False):
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd = (loss(wp) - loss(wm)) / (2 * eps)
        assert abs(fd - gw[i]) <= 1e-6 * max(1.0, abs(fd))


def test_threads_leave_every_bit_unchanged(orc):
    # the channel loops split over threads add each element's terms in the
    # serial order: the forward, the weight gradient and the input gradient
    # are bit-identical for any thread count
    B, H, W = 2, 21, 34
    rng = np.random.default_rng(12)
    w = rng.normal(scale=0.3, size=orc.param_count())
    c = rng.uniform(size=(B, H, W))
    z = rng.normal(size=(B, H, W))
    g = rng.normal(size=(B, H, W))
    ref = None
    for n in (1, 3, 7, 32):
        with orc.threads(n):
            out = (orc.policy_forward(w, c, z),) + tuple(orc.policy_backward(w, c, z, g))
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            assert np.array_equal(a, b)
    assert orc.set_threads(1) == 1
